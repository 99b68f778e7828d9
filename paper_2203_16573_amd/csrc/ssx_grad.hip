// Kernels of the misfit gradient in kappa (adjoint state of the discrete
// scheme): the pressure update of step n is p^ <- p^ + ck r^n with
// ck = dt kappa / (h Z0) and r^n = E_h h^n - D^- v^{n+1/2}, so
//   dJ/dkappa = (1 / kappa) sum_n P~^{n+1} r^n
// where P~ = ck dJ/dp^ is the transposed pressure that the adjoint sweep
// carries.  The forward sweep stores r^n for every physical cell and step
// (the fused step kernel stores it as it updates the pressure; k_grad_store
// does it after each step of the split kernels); the adjoint sweep
// accumulates P~^{n+1} r^n in FP64 before its step n.
// Only the physical grid is covered: the absorbing layer's coefficients are
// held fixed, and on the physical grid its split parts are not active.
#include "ssx_cell.h"

namespace ssx {

namespace {

// r^n = src - (dx + dz) on one group of four columns of one physical row
// and shot, with the staggered stencils and the source injection evaluated
// as in the step kernels (same weights, same accumulation order)
template <int K, typename T>
__device__ __forceinline__ void store_group(const Fields& f, const GridDims& g, int nz, int nx,
                                            const LineDev& pil, const TraceIO& pi, int gi, int iz,
                                            int shot, T* __restrict__ hist) {
  using C = typename Tr<T>::C;
  const GradRows gr(g.L, nx);
  const int I = g.L + iz, J = 4 * (gr.g0 + gi);
  const long long base = shot * g.field_stride + g.origin + (long long)I * g.pitch + J;
  const T* vx = static_cast<const T*>(f.vx) + base;
  const T* vz = static_cast<const T*>(f.vz) + base;
  C w[12];  // v_x at columns J-4 .. J+7
  ld4(*reinterpret_cast<C(*)[4]>(w), vx - 4);
  ld4(*reinterpret_cast<C(*)[4]>(w + 4), vx);
  ld4(*reinterpret_cast<C(*)[4]>(w + 8), vx + 4);
  C dx[4] = {C(0), C(0), C(0), C(0)}, dz[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
  for (int m = 1; m <= K; ++m) {
    C hi[4], lo[4];
    ld4(hi, vz + (long long)(m - 1) * g.pitch);
    ld4(lo, vz - (long long)m * g.pitch);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      dx[e] = acc(dx[e], wst<K, C>(m - 1), w[e + m + 3], w[e + 4 - m]);
      dz[e] = acc(dz[e], wst<K, C>(m - 1), hi[e], lo[e]);
    }
  }
  C r[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int Je = J + e;
    const bool phys = Je >= g.L && Je < g.L + nx;
    const C src = line_src<C, typename Tr<T>::V>(pil, pi, I, Je, shot);
    r[e] = phys ? src - (dx[e] + dz[e]) : C(0);
  }
  st4(hist + ((long long)shot * nz + iz) * gr.width() + 4 * gi, r);
}

// one thread per group of four columns of one physical row and shot
template <int K, typename T>
__global__ __launch_bounds__(256) void k_grad_store(Fields f, GridDims g, int nz, int nx,
                                                    LineDev pil, TraceIO pi, T* __restrict__ hist) {
  const int gi = blockIdx.x * 64 + threadIdx.x, iz = blockIdx.y * 4 + threadIdx.y;
  if (gi >= GradRows(g.L, nx).ng || iz >= nz) return;
  store_group<K, T>(f, g, nz, nx, pil, pi, gi, iz, blockIdx.z, hist);
}

// acc += P~ r^n over the groups of the physical rows (FP64 accumulator)
template <typename T>
__global__ __launch_bounds__(256) void k_grad_acc(Fields f, GridDims g, int nz, int nx,
                                                  const T* __restrict__ hist,
                                                  double* __restrict__ accum) {
  const GradRows gr(g.L, nx);
  const int gi = blockIdx.x * 64 + threadIdx.x, iz = blockIdx.y * 4 + threadIdx.y;
  const int shot = blockIdx.z;
  if (gi >= gr.ng || iz >= nz) return;
  const int J = 4 * (gr.g0 + gi);
  const long long o = shot * g.field_stride + g.origin + (long long)(g.L + iz) * g.pitch + J;
  const long long h = ((long long)shot * nz + iz) * gr.width() + 4 * gi;
  double p[4], r[4], a[4];
  ld4(p, static_cast<const T*>(f.p) + o);
  ld4(r, hist + h);
  ld4(a, accum + h);
#pragma unroll
  for (int e = 0; e < 4; ++e) a[e] = fma(p[e], r[e], a[e]);
  st4(accum + h, a);
}

// two steps at once: acc += P~_a r_a, then acc += P~_b r_b (the order of two
// k_grad_acc launches, a first)
template <typename T>
__global__ __launch_bounds__(256) void k_grad_acc2(Fields fa, Fields fb, GridDims g, int nz,
                                                   int nx, const T* __restrict__ ha,
                                                   const T* __restrict__ hb,
                                                   double* __restrict__ accum) {
  const GradRows gr(g.L, nx);
  const int gi = blockIdx.x * 64 + threadIdx.x, iz = blockIdx.y * 4 + threadIdx.y;
  const int shot = blockIdx.z;
  if (gi >= gr.ng || iz >= nz) return;
  const int J = 4 * (gr.g0 + gi);
  const long long o = shot * g.field_stride + g.origin + (long long)(g.L + iz) * g.pitch + J;
  const long long h = ((long long)shot * nz + iz) * gr.width() + 4 * gi;
  double pa[4], ra[4], pb[4], rb[4], a[4];
  ld4(pa, static_cast<const T*>(fa.p) + o);
  ld4(ra, ha + h);
  ld4(pb, static_cast<const T*>(fb.p) + o);
  ld4(rb, hb + h);
  ld4(a, accum + h);
#pragma unroll
  for (int e = 0; e < 4; ++e) a[e] = fma(pb[e], rb[e], fma(pa[e], ra[e], a[e]));
  st4(accum + h, a);
}

// out = acc * s / ck for every physical cell (ck = dt kappa / (h Z0), so
// with s = dt / (h Z0) this is acc / kappa); out is [shot][nz][nx]
template <typename T, typename V>
__global__ void k_grad_final(const double* __restrict__ accum, const T* __restrict__ ck,
                             GridDims g, int nz, int nx, double s, V* __restrict__ out) {
  const GradRows gr(g.L, nx);
  const int ix = blockIdx.x * blockDim.x + threadIdx.x, iz = blockIdx.y, shot = blockIdx.z;
  if (ix >= nx) return;
  const int J = g.L + ix;
  const long long o = g.origin + (long long)(g.L + iz) * g.pitch + J;
  const double a = accum[((long long)shot * nz + iz) * gr.width() + (J - 4 * gr.g0)];
  out[((long long)shot * nz + iz) * nx + ix] = V(a * s / double(ck[o]));
}

// e = a - b over n elements per shot
template <typename V>
__global__ void k_sub(const V* __restrict__ a, const V* __restrict__ b, V* __restrict__ e,
                      long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long o = (long long)blockIdx.y * n + i;
  if (i < n) e[o] = a[o] - b[o];
}

bool dims_ok(int nz, int nx, int nshots) {
  return nz > 0 && nx > 0 && nshots > 0 && nz <= 4 * 65535 && nshots <= 65535;
}
// groups: 64 groups x 4 rows per workgroup
dim3 group_grid(const GridDims& g, int nz, int nx, int nshots) {
  const GradRows gr(g.L, nx);
  return dim3((unsigned)((gr.ng + 63) / 64), (unsigned)((nz + 3) / 4), (unsigned)nshots);
}

}  // namespace

long long grad_cells(int L, int nz, int nx) { return (long long)nz * GradRows(L, nx).width(); }

hipError_t launch_grad_store(Dt dt, int order, const Fields& f, const GridDims& g, int nz, int nx,
                             const LineDev& pil, const TraceIO& pi, void* hist, int nshots,
                             hipStream_t s) {
  if (!dims_ok(nz, nx, nshots)) return hipErrorInvalidValue;
  const dim3 grid = group_grid(g, nz, nx, nshots), block(64, 4);
  if (dt == Dt::F64) {
    if (order == 8)
      hipLaunchKernelGGL((k_grad_store<4, double>), grid, block, 0, s, f, g, nz, nx, pil, pi,
                         static_cast<double*>(hist));
    else
      hipLaunchKernelGGL((k_grad_store<2, double>), grid, block, 0, s, f, g, nz, nx, pil, pi,
                         static_cast<double*>(hist));
  } else if (dt == Dt::F32) {
    if (order == 8)
      hipLaunchKernelGGL((k_grad_store<4, float>), grid, block, 0, s, f, g, nz, nx, pil, pi,
                         static_cast<float*>(hist));
    else
      hipLaunchKernelGGL((k_grad_store<2, float>), grid, block, 0, s, f, g, nz, nx, pil, pi,
                         static_cast<float*>(hist));
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_acc(Dt dt, const Fields& f, const GridDims& g, int nz, int nx,
                           const void* hist, double* acc, int nshots, hipStream_t s) {
  if (!dims_ok(nz, nx, nshots)) return hipErrorInvalidValue;
  const dim3 grid = group_grid(g, nz, nx, nshots), block(64, 4);
  if (dt == Dt::F64)
    hipLaunchKernelGGL(k_grad_acc<double>, grid, block, 0, s, f, g, nz, nx,
                       static_cast<const double*>(hist), acc);
  else if (dt == Dt::F32)
    hipLaunchKernelGGL(k_grad_acc<float>, grid, block, 0, s, f, g, nz, nx,
                       static_cast<const float*>(hist), acc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_grad_acc2(Dt dt, const Fields& fa, const Fields& fb, const GridDims& g, int nz,
                            int nx, const void* ha, const void* hb, double* acc, int nshots,
                            hipStream_t s) {
  if (!dims_ok(nz, nx, nshots)) return hipErrorInvalidValue;
  const dim3 grid = group_grid(g, nz, nx, nshots), block(64, 4);
  if (dt == Dt::F64)
    hipLaunchKernelGGL(k_grad_acc2<double>, grid, block, 0, s, fa, fb, g, nz, nx,
                       static_cast<const double*>(ha), static_cast<const double*>(hb), acc);
  else if (dt == Dt::F32)
    hipLaunchKernelGGL(k_grad_acc2<float>, grid, block, 0, s, fa, fb, g, nz, nx,
                       static_cast<const float*>(ha), static_cast<const float*>(hb), acc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_grad_final(Dt dt, const double* acc, const void* ck, const GridDims& g, int nz,
                             int nx, double scale, void* out, int nshots, hipStream_t s) {
  if (!dims_ok(nz, nx, nshots) || nz > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)nz, (unsigned)nshots);
  if (dt == Dt::F64)
    hipLaunchKernelGGL((k_grad_final<double, double>), grid, dim3(256), 0, s, acc,
                       static_cast<const double*>(ck), g, nz, nx, scale,
                       static_cast<double*>(out));
  else if (dt == Dt::F32)
    hipLaunchKernelGGL((k_grad_final<float, float>), grid, dim3(256), 0, s, acc,
                       static_cast<const float*>(ck), g, nz, nx, scale,
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
