// Vector kernels of libssx for gfx950: deterministic FP64 inner products,
// the penalty's diagonal operators, the scalar recurrences of Algorithm 1
// (preconditioned CG) and the per-shot field scale of 16-bit wavefields.
#include "ssx_device.h"

#include <cmath>
#include <mutex>

namespace ssx {

// ---------------------------------------------------------------------------
// FP64 reductions: fixed grid, fixed per-thread order, fixed wavefront
// shuffle tree, hence bitwise deterministic.

// Sums of the 256 threads of a block, written to dst[0..NV): each wavefront
// folds its 64 lanes with a fixed shuffle tree, then one thread adds the 4
// wavefront sums in a fixed order.
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double* dst) {
  static_assert(NV <= 3, "at most three sums");
  __shared__ double sh[NV][4];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    double x = acc[v];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sh[v][wave] = x;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[v] = (sh[v][0] + sh[v][1]) + (sh[v][2] + sh[v][3]);
  }
}

template <typename V, int NV>
__global__ __launch_bounds__(256) void k_dot_partial(const V* __restrict__ x,
                                                     const V* __restrict__ y, long long n,
                                                     double* partial) {
  const int shot = blockIdx.y;
  const V* xs = x + (long long)shot * n;
  const V* ys = y + (long long)shot * n;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)NBLK_DOT * 256) {
    const double a = double(xs[i]), b = double(ys[i]);
    acc[0] += a * b;
    if constexpr (NV == 3) {
      acc[1] += a * a;
      acc[2] += b * b;
    }
  }
  block_reduce_store<NV>(acc, partial + ((long long)shot * NBLK_DOT + blockIdx.x) * NV);
}

template <int NV>
__global__ __launch_bounds__(256) void k_dot_final(const double* partial, double* out,
                                                   int ostride) {
  const int shot = blockIdx.x;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    acc[v] = partial[((long long)shot * NBLK_DOT + threadIdx.x) * NV + v];
  block_reduce_store<NV>(acc, out + (long long)shot * ostride);
}

static_assert(NBLK_DOT == 256, "final reduction assumes one partial per thread");

template <int NV>
static hipError_t dot_t(bool vdbl, const void* x, const void* y, long long n, int nshots,
                        double* partial, double* out, int ostride, hipStream_t s) {
  dim3 grid(NBLK_DOT, nshots);
  if (vdbl)
    hipLaunchKernelGGL((k_dot_partial<double, NV>), grid, dim3(256), 0, s,
                       static_cast<const double*>(x), static_cast<const double*>(y), n, partial);
  else
    hipLaunchKernelGGL((k_dot_partial<float, NV>), grid, dim3(256), 0, s,
                       static_cast<const float*>(x), static_cast<const float*>(y), n, partial);
  hipLaunchKernelGGL((k_dot_final<NV>), dim3(nshots), dim3(256), 0, s, partial, out, ostride);
  return hipGetLastError();
}

hipError_t launch_dot3(bool vdbl, const void* x, const void* y, long long n, int nshots,
                       double* partial, double* out, int ostride, hipStream_t s) {
  return dot_t<3>(vdbl, x, y, n, nshots, partial, out, ostride, s);
}
hipError_t launch_dot1(bool vdbl, const void* x, const void* y, long long n, int nshots,
                       double* partial, double* out, int ostride, hipStream_t s) {
  return dot_t<1>(vdbl, x, y, n, nshots, partial, out, ostride, s);
}

// ---------------------------------------------------------------------------
// The allocation-free inner product (ssx_dot_static): its partial sums live
// in this file-scope device array, one copy per GPU, held until the process
// ends.  Every partial is written before it is read, so nothing needs
// clearing between calls; calls that overlap on one GPU share the array and
// race.
static __device__ __align__(256) double scratch[DOT_SCRATCH_SHOTS * NBLK_DOT];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};  // device address of `scratch`, per GPU
}  // namespace

// Device address of `scratch` on the current GPU, looked up once per GPU
// (the array's name in host code is only a host-side stand-in).
hipError_t dot_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_dot1_static(bool vdbl, const void* x, const void* y, long long n, int nshots,
                              double* out, hipStream_t s) {
  if (nshots < 1 || nshots > DOT_SCRATCH_SHOTS) return hipErrorInvalidValue;
  double* part = nullptr;
  hipError_t e = dot_scratch(&part);
  if (e != hipSuccess) return e;
  return dot_t<1>(vdbl, x, y, n, nshots, part, out, 1, s);
}

// ---------------------------------------------------------------------------
// diagonal operators of the penalty (lateral distance to the shot's x_s)

__device__ __forceinline__ double diag_factor(int op, double a, double dist) {
  switch (op) {
    case 0: return dist;
    case 1: return dist * dist;
    case 2: return 1.0 / sqrt(1.0 + a * a * dist * dist);
    default: return 1.0;
  }
}

template <typename V>
__global__ void k_diag(int op, double a, double s, const V* __restrict__ x, V* y, long long nt,
                       int ns, double x0, double h, const double* __restrict__ xs) {
  const int shot = blockIdx.y;
  const long long n = nt * ns;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = int(i % ns);
  const double dist = fabs(x0 + k * h - xs[shot]);
  const double fac = s * diag_factor(op, a, dist);
  const long long off = (long long)shot * n + i;
  y[off] = V(fac * double(x[off]));
}

template <typename V>
__global__ void k_add_penalty(V* q, const V* __restrict__ p, int pw,
                              const double* __restrict__ alpha2, int astride, double alpha2_host,
                              long long nt, int ns, double x0, double h,
                              const double* __restrict__ xs) {
  const int shot = blockIdx.y;
  const long long n = nt * ns;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = int(i % ns);
  const double dist = x0 + k * h - xs[shot];
  const double al2 = alpha2 ? alpha2[(long long)shot * astride] : alpha2_host;
  const double fac = pw == 2 ? al2 * dist * dist : al2 * fabs(dist);
  const long long off = (long long)shot * n + i;
  q[off] = V(double(q[off]) + fac * double(p[off]));
}

hipError_t launch_diag(bool vdbl, int op, double a, double s, const void* x, void* y,
                       long long nt, int ns, int nshots, double x0, double h,
                       const double* xs_dev, hipStream_t st) {
  const long long n = nt * ns;
  dim3 grid((unsigned)((n + 255) / 256), nshots);
  if (vdbl)
    hipLaunchKernelGGL(k_diag<double>, grid, dim3(256), 0, st, op, a, s,
                       static_cast<const double*>(x), static_cast<double*>(y), nt, ns, x0, h,
                       xs_dev);
  else
    hipLaunchKernelGGL(k_diag<float>, grid, dim3(256), 0, st, op, a, s,
                       static_cast<const float*>(x), static_cast<float*>(y), nt, ns, x0, h,
                       xs_dev);
  return hipGetLastError();
}

hipError_t launch_add_penalty(bool vdbl, void* q, const void* p, int pw, const double* alpha2,
                              int astride, double alpha2_host, long long nt, int ns,
                              int nshots, double x0, double h, const double* xs_dev,
                              hipStream_t st) {
  const long long n = nt * ns;
  dim3 grid((unsigned)((n + 255) / 256), nshots);
  if (vdbl)
    hipLaunchKernelGGL(k_add_penalty<double>, grid, dim3(256), 0, st, static_cast<double*>(q),
                       static_cast<const double*>(p), pw, alpha2, astride, alpha2_host, nt, ns,
                       x0, h, xs_dev);
  else
    hipLaunchKernelGGL(k_add_penalty<float>, grid, dim3(256), 0, st, static_cast<float*>(q),
                       static_cast<const float*>(p), pw, alpha2, astride, alpha2_host, nt, ns,
                       x0, h, xs_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Algorithm 1 scalar recurrences, one thread per shot, FP64.

__device__ __forceinline__ bool same_sign(double a, double b) { return (a > 0) == (b > 0); }

__global__ void k_pcg_init(double* sc, double alpha, int absolute, int nshots) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshots) return;
  double* c = sc + (long long)s * SC_N;
  const double dd = c[SC_DD], rr = c[SC_RR];
  const double sig = absolute ? 1.0 : (dd > 0.0 ? sqrt(rr / dd) : 0.0);
  const double al = alpha * sig;
  c[SC_ALPHA2] = al * al;
  c[SC_FLAG] = 0.0;
  c[SC_PQ0] = 0.0;
  c[SC_A] = 0.0;
  c[SC_BETA] = 0.0;
}

// k == 0: start of the iteration (g_0, r_0 known); k >= 1: after iteration k-1.
// Algorithm 1 is followed as stated: a change of sign of <g, r> or <p, q>
// (possible when M^-1 is indefinite) is recorded (flag 8) and the iteration
// goes on; only a zero or non-finite value stops a shot (its iterate is
// frozen at the last valid value).
__global__ void k_pcg_record(double* sc, double* hist, int k, int maxit, int nshots) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshots) return;
  double* c = sc + (long long)s * SC_N;
  int flag = int(c[SC_FLAG]);
  const double grn = c[SC_GRNEW];
  if (k == 0) {
    c[SC_GR] = grn;
    c[SC_GR0] = grn;
    if (!isfinite(grn)) flag |= 2;
    else if (grn == 0.0) flag |= (c[SC_RR] == 0.0 ? 4 : 1);
    c[SC_BETA] = 0.0;
  } else if ((flag & 7) == 0) {
    if (!isfinite(grn)) {
      flag |= 2;
    } else if (grn == 0.0) {
      flag |= (c[SC_RR] == 0.0 ? 4 : 1);
    } else if (!same_sign(grn, c[SC_GR0])) {
      flag |= 8;
    }
    if ((flag & 7) == 0) {
      c[SC_BETA] = grn / c[SC_GR];
      c[SC_GR] = grn;
    } else {
      c[SC_BETA] = 0.0;
    }
  } else {
    c[SC_BETA] = 0.0;
  }
  c[SC_FLAG] = double(flag);
  if (hist) {
    double* row = hist + ((long long)s * (maxit + 1) + k) * 4;
    row[0] = sqrt(c[SC_RR]);
    row[1] = sqrt(c[SC_GG]);
    row[2] = grn;
    row[3] = sqrt(c[SC_EE]);
  }
}

__global__ void k_pcg_step_length(double* sc, int nshots) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshots) return;
  double* c = sc + (long long)s * SC_N;
  int flag = int(c[SC_FLAG]);
  const double pq = c[SC_PQ];
  if ((flag & 7) == 0) {
    if (!isfinite(pq)) flag |= 2;
    else if (pq == 0.0) flag |= 1;
    else if (c[SC_PQ0] == 0.0) c[SC_PQ0] = pq;
    else if (!same_sign(pq, c[SC_PQ0])) flag |= 8;
  }
  c[SC_A] = ((flag & 7) == 0) ? c[SC_GR] / pq : 0.0;
  c[SC_FLAG] = double(flag);
}

template <typename V>
__global__ void k_pcg_update(V* h, V* r, const V* __restrict__ p, const V* __restrict__ q, V* e,
                             const V* __restrict__ Fp, long long n, long long ne,
                             const double* __restrict__ sc) {
  const int s = blockIdx.y;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double a = sc[(long long)s * SC_N + SC_A];
  if (i < n) {
    const long long o = (long long)s * n + i;
    h[o] = V(double(h[o]) + a * double(p[o]));
    r[o] = V(double(r[o]) - a * double(q[o]));
  }
  if (e != nullptr && i < ne) {
    const long long o = (long long)s * ne + i;
    e[o] = V(double(e[o]) + a * double(Fp[o]));
  }
}

template <typename V>
__global__ void k_pcg_dir(V* p, const V* __restrict__ g, long long n,
                          const double* __restrict__ sc) {
  const int s = blockIdx.y;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double b = sc[(long long)s * SC_N + SC_BETA];
  const long long o = (long long)s * n + i;
  p[o] = V(double(g[o]) + b * double(p[o]));
}

template <typename V>
__global__ void k_neg_copy(V* y, const V* __restrict__ x, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = -x[i];
}

hipError_t launch_pcg_init(double* sc, double alpha, bool absolute, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_init, dim3((nshots + 63) / 64), dim3(64), 0, s, sc, alpha,
                     (int)absolute, nshots);
  return hipGetLastError();
}
hipError_t launch_pcg_record(double* sc, double* hist, int k, int maxit, int nshots,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_record, dim3((nshots + 63) / 64), dim3(64), 0, s, sc, hist, k,
                     maxit, nshots);
  return hipGetLastError();
}
hipError_t launch_pcg_step_length(double* sc, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_step_length, dim3((nshots + 63) / 64), dim3(64), 0, s, sc, nshots);
  return hipGetLastError();
}
hipError_t launch_pcg_update(bool vdbl, void* h, void* r, const void* p, const void* q, void* e,
                             const void* Fp, long long n, long long ne, const double* sc,
                             int nshots, hipStream_t s) {
  const long long m = n > ne ? n : ne;
  dim3 grid((unsigned)((m + 255) / 256), nshots);
  if (vdbl)
    hipLaunchKernelGGL(k_pcg_update<double>, grid, dim3(256), 0, s, static_cast<double*>(h),
                       static_cast<double*>(r), static_cast<const double*>(p),
                       static_cast<const double*>(q), static_cast<double*>(e),
                       static_cast<const double*>(Fp), n, ne, sc);
  else
    hipLaunchKernelGGL(k_pcg_update<float>, grid, dim3(256), 0, s, static_cast<float*>(h),
                       static_cast<float*>(r), static_cast<const float*>(p),
                       static_cast<const float*>(q), static_cast<float*>(e),
                       static_cast<const float*>(Fp), n, ne, sc);
  return hipGetLastError();
}
hipError_t launch_pcg_dir(bool vdbl, void* p, const void* g, long long n, const double* sc,
                          int nshots, hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256), nshots);
  if (vdbl)
    hipLaunchKernelGGL(k_pcg_dir<double>, grid, dim3(256), 0, s, static_cast<double*>(p),
                       static_cast<const double*>(g), n, sc);
  else
    hipLaunchKernelGGL(k_pcg_dir<float>, grid, dim3(256), 0, s, static_cast<float*>(p),
                       static_cast<const float*>(g), n, sc);
  return hipGetLastError();
}
// ---------------------------------------------------------------------------
// per-shot power-of-two field scale from the propagation inputs (two-pass,
// no atomics)

template <typename V>
__global__ __launch_bounds__(256) void k_amax_partial(const V* __restrict__ x, double sc,
                                                      long long n, float* partial) {
  __shared__ float sh[256];
  const int shot = blockIdx.y;
  const V* xs = x + (long long)shot * n;
  float m = 0.0f;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)NBLK_DOT * 256)
    m = fmaxf(m, float(fabs(double(xs[i]) * sc)));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long long)shot * NBLK_DOT + blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_amax_final(const float* partial, int two, int nshots,
                                                    float* dyn) {
  __shared__ float sh[256];
  const int shot = blockIdx.x;
  float m = partial[(long long)shot * NBLK_DOT + threadIdx.x];
  if (two) m = fmaxf(m, partial[((long long)nshots + shot) * NBLK_DOT + threadIdx.x]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float a = sh[0];
    float s = 1.0f;
    if (a > 0.0f && isfinite(a)) {
      int e;
      frexpf(a, &e);  // a = f 2^e, f in [0.5, 1)
      s = ldexpf(1.0f, e);
    }
    dyn[shot] = s;
  }
}

hipError_t launch_field_scale(bool vdbl, const void* a, double sa, const void* b, double sb,
                              long long n, int nshots, float* partial, float* dyn,
                              hipStream_t s) {
  dim3 grid(NBLK_DOT, nshots);
  const void* xs[2] = {a, b};
  const double sc[2] = {sa, sb};
  for (int k = 0; k < (b ? 2 : 1); ++k) {
    float* part = partial + (long long)k * nshots * NBLK_DOT;
    if (vdbl)
      hipLaunchKernelGGL(k_amax_partial<double>, grid, dim3(256), 0, s,
                         static_cast<const double*>(xs[k]), sc[k], n, part);
    else
      hipLaunchKernelGGL(k_amax_partial<float>, grid, dim3(256), 0, s,
                         static_cast<const float*>(xs[k]), sc[k], n, part);
  }
  hipLaunchKernelGGL(k_amax_final, dim3(nshots), dim3(256), 0, s, partial, b ? 1 : 0, nshots,
                     dyn);
  return hipGetLastError();
}

hipError_t launch_neg_copy(bool vdbl, void* y, const void* x, long long n, hipStream_t s) {
  dim3 grid((unsigned)((n + 255) / 256));
  if (vdbl)
    hipLaunchKernelGGL(k_neg_copy<double>, grid, dim3(256), 0, s, static_cast<double*>(y),
                       static_cast<const double*>(x), n);
  else
    hipLaunchKernelGGL(k_neg_copy<float>, grid, dim3(256), 0, s, static_cast<float*>(y),
                       static_cast<const float*>(x), n);
  return hipGetLastError();
}

}  // namespace ssx
