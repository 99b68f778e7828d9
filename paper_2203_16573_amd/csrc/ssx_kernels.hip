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
// value as it will read back after a store to T
template <typename T, typename C> __device__ __forceinline__ C rnd(C v) {
  if constexpr (sizeof(T) == sizeof(C)) {
    return v;
  } else {
    T t;
    stc(&t, v);
    return ldc<C>(&t);
  }
}

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

// Per-cell update formulas, shared by every kernel variant so that all of
// them evaluate exactly the same expression (the library is built with
// -ffp-contract=off; fused multiply-adds are written out).
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// stencil difference accumulator: s + w * (hi - lo)
template <typename C> __device__ __forceinline__ C acc(C s, C w, C hi, C lo) {
  return fmac(w, hi - lo, s);
}
// velocity: a v + b cb (sgn * sum + src)
template <bool ADJ, typename C>
__device__ __forceinline__ C upd_v(C a, C b, C cb, C old, C sum, C src) {
  const C r = ADJ ? (sum + src) : (src - sum);
  return fmac(a, old, (b * cb) * r);
}
// pressure away from the absorbing frame
template <bool ADJ, typename C>
__device__ __forceinline__ C upd_p(C ck, C p, C dx, C dz, C src) {
  const C r = ADJ ? ((dx + dz) + src) : (src - (dx + dz));
  return fmac(ck, r, p);
}
// pressure in the frame; aux: forward p_x, transpose P~_x - P~_z
template <bool ADJ, typename C>
__device__ __forceinline__ C upd_p_frame(C ck, C p, C aux, C dx, C dz, C src, C axn, C bxn,
                                         C azn, C bzn, C* aux_new) {
  if constexpr (!ADJ) {
    const C px = fmac(axn, aux, -((bxn * ck) * dx));
    const C pz = fmac(azn, p - aux, (bzn * ck) * (src - dz));
    *aux_new = px;
    return px + pz;
  } else {
    const C t = (dx + dz) + src;
    const C Px = fmac(axn, p + aux, (bxn * ck) * t);
    const C Pz = fmac(azn, p, (bzn * ck) * t);
    *aux_new = Px - Pz;
    return Pz;
  }
}

constexpr int TBX = 64;  // one wavefront across x

template <typename C>
__device__ __forceinline__ C dyn_of(const TraceIO& t, int shot) {
  return t.dyn ? C(t.dyn[shot]) : C(1);
}
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
    *out = V(C(so.scale) * val * dyn_of<C>(so, shot));
  }

  C sx = C(0);
  bool split_x = false;
  if constexpr (ADJ) split_x = I < g.L || I >= g.NZ - g.L || J < g.L + K || J >= g.NX - g.L - K;
  if (!split_x) {
#pragma unroll
    for (int m = 1; m <= K; ++m)
      sx = acc(sx, wst<K, C>(m - 1), ldc<C>(p + o + m), ldc<C>(p + o + 1 - m));
  } else {
    // transposed x-split pressure P~_x = P~_z + aux, nonzero aux only in the frame
    const T* __restrict__ ax = static_cast<const T*>(f.aux) + base;
#pragma unroll
    for (int m = 1; m <= K; ++m)
      sx = acc(sx, wst<K, C>(m - 1), ldc<C>(p + o + m) + ldc<C>(ax + o + m),
               ldc<C>(p + o + 1 - m) + ldc<C>(ax + o + 1 - m));
  }
  const int NX = g.NX, NZ = g.NZ;
  const C vxn = upd_v<ADJ>(pml[2 * NX + J], pml[3 * NX + J], cb, ldc<C>(vx + o), sx, C(0));
  stc(vx + o, vxn);

  C sz = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m)
    sz = acc(sz, wst<K, C>(m - 1), ldc<C>(p + o + (long long)m * P),
             ldc<C>(p + o + (long long)(1 - m) * P));
  C src = C(0);
  if (io.n >= 0 && (I == il.row0 || I == il.row1) && J >= il.col0 && J < il.col0 + il.ntr) {
    const C w = (I == il.row0 ? C(il.w0) : C(0)) + (I == il.row1 ? C(il.w1) : C(0));
    const V* in = static_cast<const V*>(io.in) + shot * io.shot_stride + (long long)io.n * il.ntr +
                  (J - il.col0);
    src = w * (C(io.scale) * C(*in) / dyn_of<C>(io, shot));
  }
  const C vzn = upd_v<ADJ>(pml[4 * NX + 2 * NZ + I], pml[4 * NX + 3 * NZ + I], cb,
                          ldc<C>(vz + o), sz, src);
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
    *out = V(C(so.scale) * val * dyn_of<C>(so, shot));
  }

  C dx = C(0), dz = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m) {
    dx = acc(dx, wst<K, C>(m - 1), ldc<C>(vx + o + m - 1), ldc<C>(vx + o - m));
    dz = acc(dz, wst<K, C>(m - 1), ldc<C>(vz + o + (long long)(m - 1) * P),
             ldc<C>(vz + o - (long long)m * P));
  }
  C src = C(0);
  if (io.n >= 0 && (I == il.row0 || I == il.row1) && J >= il.col0 && J < il.col0 + il.ntr) {
    const C w = (I == il.row0 ? C(il.w0) : C(0)) + (I == il.row1 ? C(il.w1) : C(0));
    const V* in = static_cast<const V*>(io.in) + shot * io.shot_stride + (long long)io.n * il.ntr +
                  (J - il.col0);
    src = w * (C(io.scale) * C(*in) / dyn_of<C>(io, shot));
  }
  const int NX = g.NX, NZ = g.NZ;
  const C ck = static_cast<const C*>(cf.ck)[(long long)I * NX + J];
  const C pc = ldc<C>(p + o);
  const bool frame = I < g.L || I >= NZ - g.L || J < g.L || J >= NX - g.L;
  C pn;
  if (!frame) {
    pn = upd_p<ADJ>(ck, pc, dx, dz, src);
  } else {
    T* __restrict__ au = static_cast<T*>(f.aux) + base;
    C an;
    pn = upd_p_frame<ADJ>(ck, pc, ldc<C>(au + o), dx, dz, src, pml[J], pml[NX + J],
                          pml[4 * NX + I], pml[4 * NX + NZ + I], &an);
    stc(au + o, an);
  }
  stc(p + o, pn);
}

// ---------------------------------------------------------------------------
// Fused time step: one launch advances (p, v) by dt on a TX x TZ output tile.
//
// Phase 1 stages p^n over the tile plus a halo of R = 2K-1 cells (the
// pressure dependency radius of one full step) in LDS; the transpose also
// stages the x-split part P~_x = P~_z + aux on the tile rows when the tile
// touches the absorbing frame.  Phase 2 computes v^{n+1/2} for the tile and
// the K-cell halo the pressure stencil needs (v_x on the tile rows, v_z on
// the tile columns), writes the owned part and keeps the rest in LDS.
// Phase 3 computes p^{n+1} on the tile.  Fields are double-buffered (in ->
// out), so neighbouring tiles never see a half-updated step.  Values
// outside the grid are zero, as in the single-phase kernels.
//
// Tiles are assigned so that each XCD receives a contiguous band of tiles
// (blocks are dispatched round-robin over the 8 XCDs), which keeps halo
// re-reads inside one L2.
constexpr int TX = 64;

template <int K, bool ADJ, typename T, int TZ>
__global__ __launch_bounds__(256) void k_step(StepArgs a) {
  using C = typename Tr<T>::C;
  using V = typename Tr<T>::V;
  static_assert(TZ % 4 == 0, "tile height must be a multiple of 4");
  constexpr int R = 2 * K - 1;
  constexpr int WP = TX + 2 * R, HP = TZ + 2 * R;
  constexpr int WVX = TX + 2 * K - 1, HVZ = TZ + 2 * K - 1;
  constexpr int NP = (HP + 3) / 4;    // staging rows per thread (4 thread rows)
  constexpr int NV = TZ / 4;          // tile rows per thread
  constexpr int NVZ = (HVZ + 3) / 4;  // v_z rows per thread
  static_assert(WP <= 2 * TX && WVX <= 2 * TX, "halo wider than one extra chunk");
  __shared__ C sP[HP * WP];
  __shared__ C sPX[ADJ ? TZ * WP : 1];
  __shared__ C sVX[TZ * WVX];
  __shared__ C sVZ[HVZ * TX];

  // XCD-aware tile index
  const int nb = gridDim.x, b = blockIdx.x;
  const int full = nb >> 3, rem = nb & 7, xcd = b & 7;
  const int t = xcd * full + (xcd < rem ? xcd : rem) + (b >> 3);
  const int per_shot = a.ntx * a.ntz;
  const int shot = t / per_shot;
  const int tt = t - shot * per_shot;
  const int tzi = tt / a.ntx, txi = tt - tzi * a.ntx;
  const int x0 = txi * TX, z0 = tzi * TZ;
  const int x1 = x0 + TX, z1 = z0 + TZ;
  const int NX = a.g.NX, NZ = a.g.NZ, P = a.g.pitch, L = a.g.L;
  const long long base = a.g.origin + (long long)shot * a.g.field_stride;
  const T* __restrict__ pA = static_cast<const T*>(a.in.p) + base;
  const T* __restrict__ vxA = static_cast<const T*>(a.in.vx) + base;
  const T* __restrict__ vzA = static_cast<const T*>(a.in.vz) + base;
  const T* __restrict__ auA = static_cast<const T*>(a.in.aux) + base;
  T* __restrict__ pB = static_cast<T*>(a.out.p) + base;
  T* __restrict__ vxB = static_cast<T*>(a.out.vx) + base;
  T* __restrict__ vzB = static_cast<T*>(a.out.vz) + base;
  T* __restrict__ auB = static_cast<T*>(a.out.aux) + base;
  const C* __restrict__ pml = static_cast<const C*>(a.c.pml);
  const C* __restrict__ ckp = static_cast<const C*>(a.c.ck);
  const C cb = C(a.c.cb);
  const int lx = threadIdx.x & (TX - 1), ly = threadIdx.x >> 6;
  const bool frame_tile = (z0 < L) || (z1 > NZ - L) || (x0 < L) || (x1 > NX - L);

  // ---- issue every global load of the step before touching LDS --------
  C rp[NP][2];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int rr = ly + 4 * k, I = z0 - R + rr;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int cc = lx + TX * hh, J = x0 - R + cc;
      const bool ok = rr < HP && cc < WP && I >= 0 && I < NZ && J >= 0 && J < NX;
      rp[k][hh] = ok ? ldc<C>(pA + (long long)I * P + J) : C(0);
    }
  }
  C rvx[NV][2];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int I = z0 + ly + 4 * k;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int cc = lx + TX * hh, J = x0 - K + cc;
      const bool ok = cc < WVX && I < NZ && J >= 0 && J < NX;
      rvx[k][hh] = ok ? ldc<C>(vxA + (long long)I * P + J) : C(0);
    }
  }
  C rvz[NVZ];
#pragma unroll
  for (int k = 0; k < NVZ; ++k) {
    const int rr = ly + 4 * k, I = z0 - K + rr, J = x0 + lx;
    const bool ok = rr < HVZ && I >= 0 && I < NZ && J < NX;
    rvz[k] = ok ? ldc<C>(vzA + (long long)I * P + J) : C(0);
  }
  C rck[NV], rau[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int I = z0 + ly + 4 * k, J = x0 + lx;
    const bool ok = I < NZ && J < NX;
    rck[k] = ok ? ckp[(long long)I * NX + J] : C(0);
    const bool fr = ok && (I < L || I >= NZ - L || J < L || J >= NX - L);
    rau[k] = fr ? ldc<C>(auA + (long long)I * P + J) : C(0);
  }
  // transposed x-split part P~_x - P~_z on the tile rows (frame tiles only)
  bool use_px = false;
  C rax[ADJ ? NV : 1][2];
  if constexpr (ADJ) {
    use_px = (z0 < L) || (z1 > NZ - L) || (x0 - R < L) || (x1 + R > NX - L);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int I = z0 + ly + 4 * k;
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int cc = lx + TX * hh, J = x0 - R + cc;
        const bool ok = use_px && cc < WP && I < NZ && J >= 0 && J < NX;
        rax[k][hh] = ok ? ldc<C>(auA + (long long)I * P + J) : C(0);
      }
    }
  }

  // ---- phase 1: stage p^n (and P~_x) in LDS
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int rr = ly + 4 * k;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int cc = lx + TX * hh;
      if (rr < HP && cc < WP) sP[rr * WP + cc] = rp[k][hh];
    }
  }
  if constexpr (ADJ) {
    if (use_px) {
      // P~_x = P~_z + aux: aux goes to LDS first (its rows live in other
      // threads than the matching p rows), the sum is formed after the barrier
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int tr = ly + 4 * k;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int cc = lx + TX * hh;
          if (cc < WP) sPX[tr * WP + cc] = rax[k][hh];  // aux first; p added below
        }
      }
    }
  }
  __syncthreads();
  if constexpr (ADJ) {
    if (use_px) {
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const int tr = ly + 4 * k;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const int cc = lx + TX * hh;
          if (cc < WP) sPX[tr * WP + cc] = sP[(tr + R) * WP + cc] + sPX[tr * WP + cc];
        }
      }
      __syncthreads();
    }
  }

  // pressure-line sampling (reads p^n)
  if (a.vs.n >= 0 && a.vsl.row0 >= z0 && a.vsl.row0 < z1 && ly == 0) {
    const int J = x0 + lx;
    if (J >= a.vsl.col0 && J < a.vsl.col0 + a.vsl.ntr && J < NX) {
      const int r0 = a.vsl.row0 - z0 + R, r1 = a.vsl.row1 - z0 + R;
      const C val = C(a.vsl.w0) * sP[r0 * WP + lx + R] + C(a.vsl.w1) * sP[r1 * WP + lx + R];
      V* out = static_cast<V*>(a.vs.out) + shot * a.vs.shot_stride +
               (long long)a.vs.n * a.vsl.ntr + (J - a.vsl.col0);
      *out = V(C(a.vs.scale) * val * dyn_of<C>(a.vs, shot));
    }
  }

  // ---- phase 2a: v_x on tile rows, columns [x0 - K, x1 + K - 1)
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int rr = ly + 4 * k, I = z0 + rr;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int cc = lx + TX * hh;
      if (cc >= WVX) continue;
      const int J = x0 - K + cc;
      C val = C(0);
      if (I < NZ && J >= 0 && J < NX) {
        const C* row = (ADJ && use_px) ? (sPX + rr * WP) : (sP + (rr + R) * WP);
        const int c0 = cc - K + R;
        C sx = C(0);
#pragma unroll
        for (int m = 1; m <= K; ++m) sx = acc(sx, wst<K, C>(m - 1), row[c0 + m], row[c0 + 1 - m]);
        val = rnd<T>(upd_v<ADJ>(pml[2 * NX + J], pml[3 * NX + J], cb, rvx[k][hh], sx, C(0)));
        if (J >= x0 && J < x1) stc(vxB + (long long)I * P + J, val);
      }
      sVX[rr * WVX + cc] = val;
    }
  }
  // ---- phase 2b: v_z on tile columns, rows [z0 - K, z1 + K - 1)
#pragma unroll
  for (int k = 0; k < NVZ; ++k) {
    const int rr = ly + 4 * k;
    if (rr >= HVZ) continue;
    const int I = z0 - K + rr, J = x0 + lx;
    C val = C(0);
    if (I >= 0 && I < NZ && J < NX) {
      const int r0 = rr - K + R;
      C sz = C(0);
#pragma unroll
      for (int m = 1; m <= K; ++m)
        sz = acc(sz, wst<K, C>(m - 1), sP[(r0 + m) * WP + lx + R], sP[(r0 + 1 - m) * WP + lx + R]);
      C src = C(0);
      if (a.vi.n >= 0 && (I == a.vil.row0 || I == a.vil.row1) && J >= a.vil.col0 &&
          J < a.vil.col0 + a.vil.ntr) {
        const C w = (I == a.vil.row0 ? C(a.vil.w0) : C(0)) + (I == a.vil.row1 ? C(a.vil.w1) : C(0));
        const V* in = static_cast<const V*>(a.vi.in) + shot * a.vi.shot_stride +
                      (long long)a.vi.n * a.vil.ntr + (J - a.vil.col0);
        src = w * (C(a.vi.scale) * C(*in) / dyn_of<C>(a.vi, shot));
      }
      val = rnd<T>(upd_v<ADJ>(pml[4 * NX + 2 * NZ + I], pml[4 * NX + 3 * NZ + I], cb, rvz[k], sz,
                              src));
      if (I >= z0 && I < z1) stc(vzB + (long long)I * P + J, val);
    }
    sVZ[rr * TX + lx] = val;
  }
  __syncthreads();

  // v_z-line sampling (reads v^{n+1/2})
  if (a.ps.n >= 0 && a.psl.row0 >= z0 && a.psl.row0 < z1 && ly == 0) {
    const int J = x0 + lx;
    if (J >= a.psl.col0 && J < a.psl.col0 + a.psl.ntr && J < NX) {
      const int r0 = a.psl.row0 - z0 + K, r1 = a.psl.row1 - z0 + K;
      const C val = C(a.psl.w0) * sVZ[r0 * TX + lx] + C(a.psl.w1) * sVZ[r1 * TX + lx];
      V* out = static_cast<V*>(a.ps.out) + shot * a.ps.shot_stride +
               (long long)a.ps.n * a.psl.ntr + (J - a.psl.col0);
      *out = V(C(a.ps.scale) * val * dyn_of<C>(a.ps, shot));
    }
  }

  // ---- phase 3: p^{n+1} on the tile
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int rr = ly + 4 * k, cc = lx;
    const int I = z0 + rr, J = x0 + cc;
    if (I >= NZ || J >= NX) continue;
    C dx = C(0), dz = C(0);
#pragma unroll
    for (int m = 1; m <= K; ++m) {
      dx = acc(dx, wst<K, C>(m - 1), sVX[rr * WVX + cc + K + m - 1], sVX[rr * WVX + cc + K - m]);
      dz = acc(dz, wst<K, C>(m - 1), sVZ[(rr + K + m - 1) * TX + cc], sVZ[(rr + K - m) * TX + cc]);
    }
    C src = C(0);
    if (a.pi.n >= 0 && (I == a.pil.row0 || I == a.pil.row1) && J >= a.pil.col0 &&
        J < a.pil.col0 + a.pil.ntr) {
      const C w = (I == a.pil.row0 ? C(a.pil.w0) : C(0)) + (I == a.pil.row1 ? C(a.pil.w1) : C(0));
      const V* in = static_cast<const V*>(a.pi.in) + shot * a.pi.shot_stride +
                    (long long)a.pi.n * a.pil.ntr + (J - a.pil.col0);
      src = w * (C(a.pi.scale) * C(*in) / dyn_of<C>(a.pi, shot));
    }
    const long long o = (long long)I * P + J;
    const C ck = rck[k];
    const C pc = sP[(rr + R) * WP + cc + R];
    const bool frame = frame_tile && (I < L || I >= NZ - L || J < L || J >= NX - L);
    C pn;
    if (!frame) {
      pn = upd_p<ADJ>(ck, pc, dx, dz, src);
    } else {
      C an;
      pn = upd_p_frame<ADJ>(ck, pc, rau[k], dx, dz, src, pml[J], pml[NX + J], pml[4 * NX + I],
                            pml[4 * NX + NZ + I], &an);
      stc(auB + o, an);
    }
    stc(pB + o, pn);
  }
}

template <int K, bool ADJ, typename T>
static hipError_t step_t(int tz, const StepArgs& a, hipStream_t s) {
  const int nb = a.ntx * a.ntz * a.nshots;
  switch (tz) {
    case 8: hipLaunchKernelGGL((k_step<K, ADJ, T, 8>), dim3(nb), dim3(256), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_step<K, ADJ, T, 16>), dim3(nb), dim3(256), 0, s, a); break;
    case 32:
      if constexpr (sizeof(T) < 8) {
        hipLaunchKernelGGL((k_step<K, ADJ, T, 32>), dim3(nb), dim3(256), 0, s, a);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define SSX_DISPATCH_STEP(...)                                                   \
  do {                                                                           \
    const bool o8 = (order == 8);                                                \
    switch (dt) {                                                                \
      case Dt::F64:                                                              \
        if (o8) return adj ? step_t<4, true, double>(__VA_ARGS__) : step_t<4, false, double>(__VA_ARGS__); \
        return adj ? step_t<2, true, double>(__VA_ARGS__) : step_t<2, false, double>(__VA_ARGS__);         \
      case Dt::F32:                                                              \
        if (o8) return adj ? step_t<4, true, float>(__VA_ARGS__) : step_t<4, false, float>(__VA_ARGS__);   \
        return adj ? step_t<2, true, float>(__VA_ARGS__) : step_t<2, false, float>(__VA_ARGS__);           \
      case Dt::F16:                                                              \
        if (o8) return adj ? step_t<4, true, __half>(__VA_ARGS__) : step_t<4, false, __half>(__VA_ARGS__); \
        return adj ? step_t<2, true, __half>(__VA_ARGS__) : step_t<2, false, __half>(__VA_ARGS__);         \
      case Dt::BF16:                                                             \
        if (o8)                                                                  \
          return adj ? step_t<4, true, __hip_bfloat16>(__VA_ARGS__)             \
                     : step_t<4, false, __hip_bfloat16>(__VA_ARGS__);           \
        return adj ? step_t<2, true, __hip_bfloat16>(__VA_ARGS__)               \
                   : step_t<2, false, __hip_bfloat16>(__VA_ARGS__);             \
    }                                                                            \
    return hipErrorInvalidValue;                                                 \
  } while (0)

hipError_t launch_step(Dt dt, int order, bool adj, int tz, StepArgs a, hipStream_t s) {
  SSX_DISPATCH_STEP(tz, a, s);
}

int step_tile_width() { return TX; }

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
  *out = V(C(so.scale) * val * dyn_of<C>(so, shot));
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
