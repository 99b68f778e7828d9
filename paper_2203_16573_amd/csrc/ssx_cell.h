// Per-cell formulas of the staggered acoustic step and its transpose, and
// line injection / sampling, shared by every kernel that advances the
// wavefield, so that all of them evaluate the same expressions (the library
// is built with -ffp-contract=off; fused multiply-adds are explicit, and
// kernel variants agree bitwise).
#pragma once

#include "ssx_device.h"

namespace ssx {

// (the library is built with -ffp-contract=off; fused
// multiply-adds are explicit so every variant rounds identically)

__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

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

// stencil accumulator: s + w (hi - lo)
template <typename C> __device__ __forceinline__ C acc(C s, C w, C hi, C lo) {
  return fmac(w, hi - lo, s);
}
// velocity: a v + b cb (sgn sum + src), sgn = -1 forward, +1 transposed
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
// pressure in the frame; aux: forward p_x, transposed P~_x - P~_z
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

// absorbing-layer factors: x arrays of length pitch (origin GX), then z
// arrays of length NZ + 2 PZ (origin PZ); 1 outside the grid
template <typename C> struct Pml {
  const C* p;
  int P, NZ;
  __device__ __forceinline__ int zl() const { return NZ + 2 * PZ; }
  __device__ __forceinline__ const C* xa(int k, int J) const { return p + k * P + GX + J; }
  __device__ __forceinline__ const C* za(int k, int I) const {
    return p + 4 * P + k * zl() + PZ + I;
  }
  __device__ __forceinline__ C axn(int J) const { return p[GX + J]; }
  __device__ __forceinline__ C bxn(int J) const { return p[P + GX + J]; }
  __device__ __forceinline__ C axh(int J) const { return p[2 * P + GX + J]; }
  __device__ __forceinline__ C bxh(int J) const { return p[3 * P + GX + J]; }
  __device__ __forceinline__ C azn(int I) const { return *za(0, I); }
  __device__ __forceinline__ C bzn(int I) const { return *za(1, I); }
  __device__ __forceinline__ C azh(int I) const { return *za(2, I); }
  __device__ __forceinline__ C bzh(int I) const { return *za(3, I); }
};

template <typename C>
__device__ __forceinline__ C dyn_of(const TraceIO& t, int shot) {
  return t.dyn ? C(t.dyn[shot]) : C(1);
}

// injected value at (I, J) from a line (0 off the line)
template <typename C, typename V>
__device__ __forceinline__ C line_src(const LineDev& l, const TraceIO& io, int I, int J,
                                      int shot) {
  if (io.n < 0 || (I != l.row0 && I != l.row1) || J < l.col0 || J >= l.col0 + l.ntr) return C(0);
  const C w = (I == l.row0 ? C(l.w0) : C(0)) + (I == l.row1 ? C(l.w1) : C(0));
  const V* in = static_cast<const V*>(io.in) + shot * io.shot_stride + (long long)io.n * l.ntr +
                (J - l.col0);
  return w * (C(io.scale) * C(*in) / dyn_of<C>(io, shot));
}

template <typename C, typename V>
__device__ __forceinline__ void line_out(const LineDev& l, const TraceIO& io, int J, int shot,
                                         C val) {
  V* out = static_cast<V*>(io.out) + shot * io.shot_stride + (long long)io.n * l.ntr + (J - l.col0);
  *out = V(C(io.scale) * val * dyn_of<C>(io, shot));
}

// element i of an array, addressed as a 32-bit byte offset from a base that
// is uniform over the workgroup (one scalar base + one vector offset)
template <typename T> __device__ __forceinline__ const T* at(const T* b, unsigned i) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(b) + i * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ T* at(T* b, unsigned i) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(b) + i * (unsigned)sizeof(T));
}

template <typename C, typename V>
__device__ __forceinline__ C line_src_at(const LineDev& l, const TraceIO& io, int idx, int nt,
                                         int I, int J, int shot) {
  if (!io.in || idx < 0 || idx >= nt || (I != l.row0 && I != l.row1) || J < l.col0 ||
      J >= l.col0 + l.ntr)
    return C(0);
  const C w = (I == l.row0 ? C(l.w0) : C(0)) + (I == l.row1 ? C(l.w1) : C(0));
  const V* in = static_cast<const V*>(io.in) + shot * io.shot_stride + (long long)idx * l.ntr +
                (J - l.col0);
  return w * (C(io.scale) * C(*in) / dyn_of<C>(io, shot));
}

template <typename C, typename V>
__device__ __forceinline__ void line_out_at(const LineDev& l, const TraceIO& io, int idx, int J,
                                            int shot, C val) {
  V* out = static_cast<V*>(io.out) + shot * io.shot_stride + (long long)idx * l.ntr + (J - l.col0);
  *out = V(C(io.scale) * val * dyn_of<C>(io, shot));
}

}  // namespace ssx
