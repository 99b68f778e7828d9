// HIP kernels for gfx950 (CDNA4): staggered-grid acoustic time step and its
// exact transpose, fused line injection / sampling, and the FP64 Krylov
// reductions of Algorithm 1.
//
// Scheme (Numerical Examples, "Synthetic models and simulation": staggered
// grid, order 2 in time and 2K in space, PML on all sides, linear
// interpolation for sampling, its transpose for injection).  Stored
// variables are scaled: p^ = p / Z0 and v^ = v with Z0 a reference
// impedance, so that both update coefficients are Courant-sized:
//   cb = Z0 dt / (rho h),  ck = dt kappa / (h Z0).
//
// Forward step n (two launches):
//   vel:  v_x <- a v_x - b cb Dx+ p ;  v_z <- a v_z + b cb (-Dz+ p + w f[n])
//   pres: p   <- p + ck (-(Dx- v_x + Dz- v_z) + w h[n])      (interior)
//         split p = p_x + p_z in the absorbing frame, with p_x stored.
// Transposed step n (scaled adjoint variables P~ = ck b' pbar,
// V~ = b cb vbar; interior P~_x = P~_z): the same two launches with the
// sign of the stencil terms flipped, the x-stencil of vel reading P~_x and
// the z-stencil P~_z, and pres adding the full divergence to both split
// components (the transpose exchanges which side of the update is split).
//
// Sampling is fused into the launch that reads the sampled field without
// writing it: vel samples pressure lines, pres samples v_z lines.
#include "ssx_internal.h"

#include <cmath>

namespace ssx {

template <typename T> struct Tr;
template <> struct Tr<double> { using C = double; using V = double; };
template <> struct Tr<float> { using C = float; using V = float; };
template <> struct Tr<__half> { using C = float; using V = float; };
template <> struct Tr<__hip_bfloat16> { using C = float; using V = float; };

template <typename C> __device__ __forceinline__ C ldc(const double* p) { return C(*p); }
template <typename C> __device__ __forceinline__ C ldc(const float* p) { return C(*p); }
template <typename C> __device__ __forceinline__ C ldc(const __half* p) {
  return C(__half2float(*p));
}
template <typename C> __device__ __forceinline__ C ldc(const __hip_bfloat16* p) {
  return C(__bfloat162float(*p));
}
__device__ __forceinline__ void stc(double* p, double v) { *p = v; }
__device__ __forceinline__ void stc(float* p, float v) { *p = v; }
__device__ __forceinline__ void stc(__half* p, float v) { *p = __float2half(v); }
__device__ __forceinline__ void stc(__hip_bfloat16* p, float v) { *p = __float2bfloat16(v); }

// Staggered first-derivative weights c_1..c_K (Taylor / Fornberg).
template <int K, typename C> __device__ __forceinline__ C wst(int m) {
  if constexpr (K == 2) {
    return m == 0 ? C(9.0 / 8.0) : C(-1.0 / 24.0);
  } else {
    return m == 0   ? C(1225.0 / 1024.0)
           : m == 1 ? C(-245.0 / 3072.0)
           : m == 2 ? C(49.0 / 5120.0)
                    : C(-5.0 / 7168.0);
  }
}

constexpr int TBX = 64;  // one wavefront across x
constexpr int TBY = 4;

// ---------------------------------------------------------------------------
// velocity update (+ pressure-line sampling, + v_z injection)
template <int K, bool ADJ, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_vel(Fields f, GridDims g, Coef cf,
                                                  LineDev sl, TraceIO so, LineDev il,
                                                  TraceIO io) {
  using C = typename Tr<T>::C;
  using V = typename Tr<T>::V;
  const int J = blockIdx.x * TBX + threadIdx.x;
  const int I = blockIdx.y * TBY + threadIdx.y;
  const int shot = blockIdx.z;
  if (I >= g.NZ || J >= g.NX) return;
  const long long base = g.origin + (long long)shot * g.field_stride;
  const T* __restrict__ p = static_cast<const T*>(f.p) + base;
  T* __restrict__ vx = static_cast<T*>(f.vx) + base;
  T* __restrict__ vz = static_cast<T*>(f.vz) + base;
  const int P = g.pitch;
  const long long o = (long long)I * P + J;
  const C* __restrict__ pml = static_cast<const C*>(cf.pml);
  const C cb = C(cf.cb);

  if (so.n >= 0 && I == sl.row0 && J >= sl.col0 && J < sl.col0 + sl.ntr) {
    const C val = C(sl.w0) * ldc<C>(p + o) + C(sl.w1) * ldc<C>(p + (long long)sl.row1 * P + J);
    V* out = static_cast<V*>(so.out) + shot * so.shot_stride + (long long)so.n * sl.ntr +
             (J - sl.col0);
    *out = V(C(so.scale) * val);
  }

  C sx = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m) sx += wst<K, C>(m - 1) * (ldc<C>(p + o + m) - ldc<C>(p + o + 1 - m));
  if constexpr (ADJ) {
    // x-split part of the transposed pressure, nonzero only in the frame
    if (I < g.L || I >= g.NZ - g.L || J < g.L + K || J >= g.NX - g.L - K) {
      const T* __restrict__ ax = static_cast<const T*>(f.aux) + base;
#pragma unroll
      for (int m = 1; m <= K; ++m)
        sx += wst<K, C>(m - 1) * (ldc<C>(ax + o + m) - ldc<C>(ax + o + 1 - m));
    }
  }
  constexpr C sgn = ADJ ? C(1) : C(-1);
  const int NX = g.NX, NZ = g.NZ;
  const C vxn = pml[2 * NX + J] * ldc<C>(vx + o) + pml[3 * NX + J] * cb * (sgn * sx);
  stc(vx + o, vxn);

  C sz = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m)
    sz += wst<K, C>(m - 1) * (ldc<C>(p + o + (long long)m * P) - ldc<C>(p + o + (long long)(1 - m) * P));
  C src = C(0);
  if (io.n >= 0 && (I == il.row0 || I == il.row1) && J >= il.col0 && J < il.col0 + il.ntr) {
    const C w = (I == il.row0 ? C(il.w0) : C(0)) + (I == il.row1 ? C(il.w1) : C(0));
    const V* in = static_cast<const V*>(io.in) + shot * io.shot_stride + (long long)io.n * il.ntr +
                  (J - il.col0);
    src = w * (C(io.scale) * C(*in));
  }
  const C vzn = pml[4 * NX + 2 * NZ + I] * ldc<C>(vz + o) +
                pml[4 * NX + 3 * NZ + I] * cb * (sgn * sz + src);
  stc(vz + o, vzn);
}

// ---------------------------------------------------------------------------
// pressure update (+ v_z-line sampling, + pressure injection)
template <int K, bool ADJ, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_pres(Fields f, GridDims g, Coef cf,
                                                   LineDev sl, TraceIO so, LineDev il,
                                                   TraceIO io) {
  using C = typename Tr<T>::C;
  using V = typename Tr<T>::V;
  const int J = blockIdx.x * TBX + threadIdx.x;
  const int I = blockIdx.y * TBY + threadIdx.y;
  const int shot = blockIdx.z;
  if (I >= g.NZ || J >= g.NX) return;
  const long long base = g.origin + (long long)shot * g.field_stride;
  T* __restrict__ p = static_cast<T*>(f.p) + base;
  const T* __restrict__ vx = static_cast<const T*>(f.vx) + base;
  const T* __restrict__ vz = static_cast<const T*>(f.vz) + base;
  const int P = g.pitch;
  const long long o = (long long)I * P + J;
  const C* __restrict__ pml = static_cast<const C*>(cf.pml);

  if (so.n >= 0 && I == sl.row0 && J >= sl.col0 && J < sl.col0 + sl.ntr) {
    const C val =
        C(sl.w0) * ldc<C>(vz + o) + C(sl.w1) * ldc<C>(vz + (long long)sl.row1 * P + J);
    V* out = static_cast<V*>(so.out) + shot * so.shot_stride + (long long)so.n * sl.ntr +
             (J - sl.col0);
    *out = V(C(so.scale) * val);
  }

  C dx = C(0), dz = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m) {
    dx += wst<K, C>(m - 1) * (ldc<C>(vx + o + m - 1) - ldc<C>(vx + o - m));
    dz += wst<K, C>(m - 1) *
          (ldc<C>(vz + o + (long long)(m - 1) * P) - ldc<C>(vz + o - (long long)m * P));
  }
  C src = C(0);
  if (io.n >= 0 && (I == il.row0 || I == il.row1) && J >= il.col0 && J < il.col0 + il.ntr) {
    const C w = (I == il.row0 ? C(il.w0) : C(0)) + (I == il.row1 ? C(il.w1) : C(0));
    const V* in = static_cast<const V*>(io.in) + shot * io.shot_stride + (long long)io.n * il.ntr +
                  (J - il.col0);
    src = w * (C(io.scale) * C(*in));
  }
  const int NX = g.NX, NZ = g.NZ;
  const C ck = static_cast<const C*>(cf.ck)[(long long)I * NX + J];
  const C pc = ldc<C>(p + o);
  const bool frame = I < g.L || I >= NZ - g.L || J < g.L || J >= NX - g.L;
  C pn;
  if (!frame) {
    if constexpr (ADJ)
      pn = pc + ck * ((dx + dz) + src);
    else
      pn = pc + ck * (src - (dx + dz));
  } else {
    T* __restrict__ au = static_cast<T*>(f.aux) + base;
    const C axn = pml[J], bxn = pml[NX + J];
    const C azn = pml[4 * NX + I], bzn = pml[4 * NX + NZ + I];
    if constexpr (!ADJ) {
      C px = ldc<C>(au + o);
      C pz = pc - px;
      px = axn * px - bxn * ck * dx;
      pz = azn * pz + bzn * ck * (src - dz);
      pn = px + pz;
      stc(au + o, px);
    } else {
      const C t = (dx + dz) + src;
      const C Px = axn * (pc + ldc<C>(au + o)) + bxn * ck * t;
      const C Pz = azn * pc + bzn * ck * t;
      pn = Pz;
      stc(au + o, Px - Pz);
    }
  }
  stc(p + o, pn);
}

template <typename T>
__global__ void k_sample_p(Fields f, GridDims g, LineDev sl, TraceIO so) {
  using C = typename Tr<T>::C;
  using V = typename Tr<T>::V;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int shot = blockIdx.y;
  if (k >= sl.ntr) return;
  const long long base = g.origin + (long long)shot * g.field_stride;
  const T* p = static_cast<const T*>(f.p) + base;
  const int J = sl.col0 + k;
  const C val = C(sl.w0) * ldc<C>(p + (long long)sl.row0 * g.pitch + J) +
                C(sl.w1) * ldc<C>(p + (long long)sl.row1 * g.pitch + J);
  V* out = static_cast<V*>(so.out) + shot * so.shot_stride + (long long)so.n * sl.ntr + k;
  *out = V(C(so.scale) * val);
}

__global__ void k_zero(uint32_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// ---------------------------------------------------------------------------
// launchers

template <int K, bool ADJ, typename T>
static hipError_t vel_t(const Fields& f, const GridDims& g, const Coef& c, const LineDev& sl,
                        const TraceIO& so, const LineDev& il, const TraceIO& io, int ns,
                        hipStream_t s) {
  dim3 grid((g.NX + TBX - 1) / TBX, (g.NZ + TBY - 1) / TBY, ns);
  hipLaunchKernelGGL((k_vel<K, ADJ, T>), grid, dim3(TBX, TBY), 0, s, f, g, c, sl, so, il, io);
  return hipGetLastError();
}
template <int K, bool ADJ, typename T>
static hipError_t pres_t(const Fields& f, const GridDims& g, const Coef& c, const LineDev& sl,
                         const TraceIO& so, const LineDev& il, const TraceIO& io, int ns,
                         hipStream_t s) {
  dim3 grid((g.NX + TBX - 1) / TBX, (g.NZ + TBY - 1) / TBY, ns);
  hipLaunchKernelGGL((k_pres<K, ADJ, T>), grid, dim3(TBX, TBY), 0, s, f, g, c, sl, so, il, io);
  return hipGetLastError();
}

#define SSX_DISPATCH(FN, ...)                                                    \
  do {                                                                           \
    const bool o8 = (order == 8);                                                \
    switch (dt) {                                                                \
      case Dt::F64:                                                              \
        if (o8) return adj ? FN<4, true, double>(__VA_ARGS__) : FN<4, false, double>(__VA_ARGS__); \
        return adj ? FN<2, true, double>(__VA_ARGS__) : FN<2, false, double>(__VA_ARGS__);         \
      case Dt::F32:                                                              \
        if (o8) return adj ? FN<4, true, float>(__VA_ARGS__) : FN<4, false, float>(__VA_ARGS__);   \
        return adj ? FN<2, true, float>(__VA_ARGS__) : FN<2, false, float>(__VA_ARGS__);           \
      case Dt::F16:                                                              \
        if (o8) return adj ? FN<4, true, __half>(__VA_ARGS__) : FN<4, false, __half>(__VA_ARGS__); \
        return adj ? FN<2, true, __half>(__VA_ARGS__) : FN<2, false, __half>(__VA_ARGS__);         \
      case Dt::BF16:                                                             \
        if (o8)                                                                  \
          return adj ? FN<4, true, __hip_bfloat16>(__VA_ARGS__)                 \
                     : FN<4, false, __hip_bfloat16>(__VA_ARGS__);               \
        return adj ? FN<2, true, __hip_bfloat16>(__VA_ARGS__)                   \
                   : FN<2, false, __hip_bfloat16>(__VA_ARGS__);                 \
    }                                                                            \
    return hipErrorInvalidValue;                                                 \
  } while (0)

hipError_t launch_vel(Dt dt, int order, bool adj, const Fields& f, const GridDims& g,
                      const Coef& c, const LineDev& sl, const TraceIO& so, const LineDev& il,
                      const TraceIO& io, int nshots, hipStream_t s) {
  SSX_DISPATCH(vel_t, f, g, c, sl, so, il, io, nshots, s);
}

hipError_t launch_pres(Dt dt, int order, bool adj, const Fields& f, const GridDims& g,
                       const Coef& c, const LineDev& sl, const TraceIO& so, const LineDev& il,
                       const TraceIO& io, int nshots, hipStream_t s) {
  SSX_DISPATCH(pres_t, f, g, c, sl, so, il, io, nshots, s);
}

hipError_t launch_sample_p(Dt dt, const Fields& f, const GridDims& g, const LineDev& line,
                           const TraceIO& io, int nshots, hipStream_t s) {
  dim3 grid((line.ntr + 255) / 256, nshots);
  switch (dt) {
    case Dt::F64: hipLaunchKernelGGL(k_sample_p<double>, grid, dim3(256), 0, s, f, g, line, io); break;
    case Dt::F32: hipLaunchKernelGGL(k_sample_p<float>, grid, dim3(256), 0, s, f, g, line, io); break;
    case Dt::F16: hipLaunchKernelGGL(k_sample_p<__half>, grid, dim3(256), 0, s, f, g, line, io); break;
    case Dt::BF16:
      hipLaunchKernelGGL(k_sample_p<__hip_bfloat16>, grid, dim3(256), 0, s, f, g, line, io);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_zero(void* ptr, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  if (n == 0) return hipSuccess;
  size_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<uint32_t*>(ptr), n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 reductions: fixed grid and fixed tree, hence bitwise deterministic.

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double* dst) {
  __shared__ double sh[NV][256];
  const int t = threadIdx.x;
#pragma unroll
  for (int v = 0; v < NV; ++v) sh[v][t] = acc[v];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sh[v][t] += sh[v][t + w];
    }
    __syncthreads();
  }
  if (t == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) dst[v] = sh[v][0];
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
__global__ void k_add_penalty(V* q, const V* __restrict__ p, const double* __restrict__ alpha2,
                              int astride, double alpha2_host, long long nt, int ns, double x0,
                              double h, const double* __restrict__ xs) {
  const int shot = blockIdx.y;
  const long long n = nt * ns;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = int(i % ns);
  const double dist = x0 + k * h - xs[shot];
  const double al2 = alpha2 ? alpha2[(long long)shot * astride] : alpha2_host;
  const double fac = al2 * dist * dist;
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

hipError_t launch_add_penalty(bool vdbl, void* q, const void* p, const double* alpha2,
                              int astride, double alpha2_host, long long nt, int ns,
                              int nshots, double x0, double h, const double* xs_dev,
                              hipStream_t st) {
  const long long n = nt * ns;
  dim3 grid((unsigned)((n + 255) / 256), nshots);
  if (vdbl)
    hipLaunchKernelGGL(k_add_penalty<double>, grid, dim3(256), 0, st, static_cast<double*>(q),
                       static_cast<const double*>(p), alpha2, astride, alpha2_host, nt, ns, x0,
                       h, xs_dev);
  else
    hipLaunchKernelGGL(k_add_penalty<float>, grid, dim3(256), 0, st, static_cast<float*>(q),
                       static_cast<const float*>(p), alpha2, astride, alpha2_host, nt, ns, x0,
                       h, xs_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Algorithm 1 scalar recurrences, one thread per shot, FP64.

__device__ __forceinline__ bool same_sign(double a, double b) { return (a > 0) == (b > 0); }

__global__ void k_pcg_init(double* sc, double alpha_rel, int nshots) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nshots) return;
  double* c = sc + (long long)s * SC_N;
  const double dd = c[SC_DD], rr = c[SC_RR];
  const double sig = dd > 0.0 ? sqrt(rr / dd) : 0.0;
  const double al = alpha_rel * sig;
  c[SC_ALPHA2] = al * al;
  c[SC_FLAG] = 0.0;
  c[SC_PQ0] = 0.0;
  c[SC_A] = 0.0;
  c[SC_BETA] = 0.0;
}

// k == 0: start of the iteration (g_0, r_0 known); k >= 1: after iteration k-1.
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
  } else if (flag == 0) {
    if (!isfinite(grn)) {
      flag |= 2;
    } else if (grn == 0.0) {
      flag |= (c[SC_RR] == 0.0 ? 4 : 1);
    } else if (!same_sign(grn, c[SC_GR0])) {
      flag |= 1;
    }
    if (flag == 0) {
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
  if (flag == 0) {
    if (!isfinite(pq)) flag |= 2;
    else if (pq == 0.0) flag |= 1;
    else if (c[SC_PQ0] == 0.0) c[SC_PQ0] = pq;
    else if (!same_sign(pq, c[SC_PQ0])) flag |= 1;
  }
  c[SC_A] = (flag == 0) ? c[SC_GR] / pq : 0.0;
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

hipError_t launch_pcg_init(double* sc, double alpha_rel, int nshots, hipStream_t s) {
  hipLaunchKernelGGL(k_pcg_init, dim3((nshots + 63) / 64), dim3(64), 0, s, sc, alpha_rel,
                     nshots);
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
