// Internal interface between the host side of the 3D entry points
// (ssx3_api.cpp) and their kernels (ssx3.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace ssx3 {

struct Dims3 {
  int NZ, NY, NX;  // padded grid: physical + 2 npml per axis
  int L;           // absorbing cells per side
};

// A plane of traces: grid rows r0 (weight w0) and r1 (weight w1; r1 < 0:
// one row), lateral node ranges [y0, y0 + ny) and [x0, x0 + nx); trace
// index (y - y0) * nx + (x - x0).
struct Plane3 {
  int r0, r1;
  double w0, w1;
  int y0, ny, x0, nx;
};

// The NFIELDS3 [NZ][NY][NX] fields, carved from one buffer in this order.
// The pressure parts px, py, pz are used in the absorbing frame only; p
// holds the total pressure everywhere (forward) or, in the transposed
// sweep, the common value of the three parts' adjoints off the frame
// (equal there: they receive the same updates).  qx, qy, qz (transposed
// sweep only): b_node,a ck times the adjoint of pressure part a, and ux,
// uy, uz: b_half,a cb times the adjoint of v_a, each stored by the kernel
// that updates that adjoint, so that the next kernel reads one value per
// stencil neighbour.
constexpr int NFIELDS3 = 13;
template <typename T>
struct Fields3 {
  T *vx, *vy, *vz, *px, *py, *pz, *p, *qx, *qy, *qz, *ux, *uy, *uz;
};
template <typename T>
inline Fields3<T> fields3(const void* base, const Dims3& d) {
  T* b = static_cast<T*>(const_cast<void*>(base));
  const long long n = (long long)d.NZ * d.NY * d.NX;
  return {b,         b + n,     b + 2 * n, b + 3 * n, b + 4 * n,  b + 5 * n, b + 6 * n,
          b + 7 * n, b + 8 * n, b + 9 * n, b + 10 * n, b + 11 * n, b + 12 * n};
}

// One time step of the fields.  Forward: v then p, with the pressure
// source plane pl and its samples tr, and the normal-load plane pl2 (v_z
// nodes) and its samples tr2 (either null: none).  Transposed: the velocity
// and pressure adjoints, with the pressure recording of the next-lower step
// (pl, tr) and this step's v_z recording (pl2, tr2).  fac: the layer
// factors, per axis z, y, x four arrays a_node, b_node, a_half, b_half; ck =
// dt kappa / h per cell; cb = dt / (rho h).
hipError_t launch3_step(bool f64, int order, bool adj, const void* fields, const Dims3& d,
                        const void* fac, const void* ck, double cb, const Plane3& pl,
                        const void* tr, const Plane3& pl2, const void* tr2, hipStream_t s);
// each pressure part's adjoint += R^T tr on plane pl (and its q updated)
hipError_t launch3_spread(bool f64, const void* fields, const Dims3& d, const Plane3& pl,
                          const void* fac, const void* ck, const void* tr, hipStream_t s);
// out = R v on plane pl: mode 0 v = p; 1 (transposed sweep) v = b_node,z ck
// times the adjoint of the pressure's z part; 2 v = v_z; 3 (transposed
// sweep) v = b_half,z cb times v_z's adjoint
hipError_t launch3_gather(bool f64, int mode, const void* fields, const Dims3& d,
                          const Plane3& pl, const void* fac, const void* ck, double cb,
                          void* out, hipStream_t s);
// y = sc s_t x per trace t (n values, ntr traces per step): s_t = dist_t
// (op 0), dist_t^2 (op 1), (1 + a^2 dist_t^2)^(-1/2) (op 2)
hipError_t launch3_diag(bool f64, int op, double a, double sc, const double* dist, const void* x,
                        void* y, long long n, int ntr, hipStream_t s);
// y = x + a z
hipError_t launch3_axpy(bool f64, void* y, const void* x, double a, const void* z, long long n,
                        hipStream_t s);

// out[0] = <x, y> in FP64 over n values (partial: device double[256])
hipError_t launch3_dot(bool f64, const void* x, const void* y, long long n, double* partial,
                       double* out, hipStream_t s);

}  // namespace ssx3
