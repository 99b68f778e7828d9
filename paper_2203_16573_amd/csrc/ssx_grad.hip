// Kernels of the misfit gradient in kappa (adjoint state of the discrete
// scheme): the pressure update of step n is p^ <- p^ + ck r^n with
// ck = dt kappa / (h Z0) and r^n = E_h h^n - D^- v^{n+1/2}, so
//   dJ/dkappa = (1 / kappa) sum_n P~^{n+1} r^n
// where P~ = ck dJ/dp^ is the transposed pressure that the adjoint sweep
// carries.  The forward sweep stores r^n for every physical cell and step;
// the adjoint sweep accumulates P~^{n+1} r^n in FP64 before its step n.
// Only the physical grid is covered: the absorbing layer's coefficients are
// held fixed, and on the physical grid its split parts are not active.
#include "ssx_cell.h"

namespace ssx {

namespace {

// one thread per physical cell of one shot: r^n = src - (dx + dz) with the
// staggered stencils and the source injection evaluated as in the step
// kernels (same weights, same accumulation order)
template <int K, typename T>
__global__ void k_grad_store(Fields f, GridDims g, int nz, int nx, LineDev pil, TraceIO pi,
                             T* __restrict__ hist, long long shot_cells) {
  using C = typename Tr<T>::C;
  const int shot = blockIdx.y;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nz * nx) return;
  const int iz = int(i / nx), ix = int(i - (long long)iz * nx);
  const int I = g.L + iz, J = g.L + ix;
  const long long base = shot * g.field_stride + g.origin + (long long)I * g.pitch + J;
  const T* vx = static_cast<const T*>(f.vx) + base;
  const T* vz = static_cast<const T*>(f.vz) + base;
  C dx = C(0), dz = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m) {
    dx = acc(dx, wst<K, C>(m - 1), ldc<C>(vx + (m - 1)), ldc<C>(vx - m));
    dz = acc(dz, wst<K, C>(m - 1), ldc<C>(vz + (long long)(m - 1) * g.pitch),
             ldc<C>(vz - (long long)m * g.pitch));
  }
  const C src = line_src<C, typename Tr<T>::V>(pil, pi, I, J, shot);
  hist[shot * shot_cells + i] = T(src - (dx + dz));
}

// acc += P~ r^n for every physical cell (FP64 accumulator)
template <typename T>
__global__ void k_grad_acc(Fields f, GridDims g, int nz, int nx, const T* __restrict__ hist,
                           long long shot_cells, double* __restrict__ acc) {
  const int shot = blockIdx.y;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nz * nx) return;
  const int iz = int(i / nx), ix = int(i - (long long)iz * nx);
  const long long o = shot * g.field_stride + g.origin + (long long)(g.L + iz) * g.pitch + g.L + ix;
  const double p = double(static_cast<const T*>(f.p)[o]);
  const double r = double(hist[shot * shot_cells + i]);
  double* a = acc + shot * shot_cells + i;
  *a = fma(p, r, *a);
}

// out = acc * s / ck for every physical cell (ck = dt kappa / (h Z0), so
// with s = dt / (h Z0) this is acc / kappa)
template <typename T, typename V>
__global__ void k_grad_final(const double* __restrict__ acc, const T* __restrict__ ck,
                             GridDims g, int nz, int nx, double s, long long shot_cells,
                             V* __restrict__ out) {
  const int shot = blockIdx.y;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)nz * nx) return;
  const int iz = int(i / nx), ix = int(i - (long long)iz * nx);
  const long long o = g.origin + (long long)(g.L + iz) * g.pitch + g.L + ix;
  out[shot * shot_cells + i] = V(acc[shot * shot_cells + i] * s / double(ck[o]));
}

// e = a - b over n elements per shot
template <typename V>
__global__ void k_sub(const V* __restrict__ a, const V* __restrict__ b, V* __restrict__ e,
                      long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long o = (long long)blockIdx.y * n + i;
  if (i < n) e[o] = a[o] - b[o];
}

dim3 cells_grid(int nz, int nx, int nshots) {
  return dim3((unsigned)(((long long)nz * nx + 255) / 256), nshots);
}

}  // namespace

hipError_t launch_grad_store(Dt dt, int order, const Fields& f, const GridDims& g, int nz, int nx,
                             const LineDev& pil, const TraceIO& pi, void* hist, int nshots,
                             hipStream_t s) {
  const long long sc = (long long)nz * nx;
  const dim3 grid = cells_grid(nz, nx, nshots);
  if (dt == Dt::F64) {
    if (order == 8)
      hipLaunchKernelGGL((k_grad_store<4, double>), grid, dim3(256), 0, s, f, g, nz, nx, pil, pi,
                         static_cast<double*>(hist), sc);
    else
      hipLaunchKernelGGL((k_grad_store<2, double>), grid, dim3(256), 0, s, f, g, nz, nx, pil, pi,
                         static_cast<double*>(hist), sc);
  } else if (dt == Dt::F32) {
    if (order == 8)
      hipLaunchKernelGGL((k_grad_store<4, float>), grid, dim3(256), 0, s, f, g, nz, nx, pil, pi,
                         static_cast<float*>(hist), sc);
    else
      hipLaunchKernelGGL((k_grad_store<2, float>), grid, dim3(256), 0, s, f, g, nz, nx, pil, pi,
                         static_cast<float*>(hist), sc);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_acc(Dt dt, const Fields& f, const GridDims& g, int nz, int nx,
                           const void* hist, double* acc, int nshots, hipStream_t s) {
  const long long sc = (long long)nz * nx;
  const dim3 grid = cells_grid(nz, nx, nshots);
  if (dt == Dt::F64)
    hipLaunchKernelGGL(k_grad_acc<double>, grid, dim3(256), 0, s, f, g, nz, nx,
                       static_cast<const double*>(hist), sc, acc);
  else if (dt == Dt::F32)
    hipLaunchKernelGGL(k_grad_acc<float>, grid, dim3(256), 0, s, f, g, nz, nx,
                       static_cast<const float*>(hist), sc, acc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_grad_final(Dt dt, const double* acc, const void* ck, const GridDims& g, int nz,
                             int nx, double scale, void* out, int nshots, hipStream_t s) {
  const long long sc = (long long)nz * nx;
  const dim3 grid = cells_grid(nz, nx, nshots);
  if (dt == Dt::F64)
    hipLaunchKernelGGL((k_grad_final<double, double>), grid, dim3(256), 0, s, acc,
                       static_cast<const double*>(ck), g, nz, nx, scale, sc,
                       static_cast<double*>(out));
  else if (dt == Dt::F32)
    hipLaunchKernelGGL((k_grad_final<float, float>), grid, dim3(256), 0, s, acc,
                       static_cast<const float*>(ck), g, nz, nx, scale, sc,
                       static_cast<float*>(out));
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sub(bool vdbl, const void* a, const void* b, void* e, long long n, int nshots,
                      hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256), nshots);
  if (vdbl)
    hipLaunchKernelGGL(k_sub<double>, grid, dim3(256), 0, s, static_cast<const double*>(a),
                       static_cast<const double*>(b), static_cast<double*>(e), n);
  else
    hipLaunchKernelGGL(k_sub<float>, grid, dim3(256), 0, s, static_cast<const float*>(a),
                       static_cast<const float*>(b), static_cast<float*>(e), n);
  return hipGetLastError();
}

}  // namespace ssx
