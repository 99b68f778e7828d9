// HIP stencil kernels for gfx950 (CDNA4): the staggered-grid acoustic time
// step and its exact transpose, with line injection and sampling fused in.
//
// Scheme (Numerical Examples, "Synthetic models and simulation": staggered
// grid, order 2 in time and 2K in space, PML on all sides, linear
// interpolation for sampling, its transpose for injection).  Stored
// variables are scaled, p^ = p / Z0 and v^ = v with Z0 a reference
// impedance, so that both update coefficients are Courant-sized:
//   cb = Z0 dt / (rho h),  ck = dt kappa / (h Z0).
//
// Forward step n:
//   v_x <- a v_x - b cb Dx+ p ;  v_z <- a v_z + b cb (-Dz+ p + w f[n])
//   p   <- p + ck (-(Dx- v_x + Dz- v_z) + w h[n])               (interior)
//   in the absorbing frame p = p_x + p_z is split, with p_x stored.
// Transposed step n (scaled adjoint variables P~ = ck b' pbar,
// V~ = b cb vbar; interior P~_x = P~_z): the stencil terms change sign, the
// x-stencil of the velocity update reads P~_x and the z-stencil P~_z, and
// both split pressure parts receive the full divergence (transposition
// exchanges which side of the update is split).
//
// Two implementations compute the same expressions (bitwise equal for every
// storage type): k_vel + k_pres, one thread per cell and two launches per
// step (the reference); and k_step, one launch per step on an LDS-staged
// tile with each thread owning 1 x 4 cells.
#include "ssx_cell.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

namespace ssx {

constexpr int TBX = 64;  // split kernels: one wavefront across x
constexpr int TBY = 4;

// ---------------------------------------------------------------------------
// split reference kernels: velocity update (+ pressure-line sampling, +
// v_z injection), then pressure update (+ v_z-line sampling, + pressure
// injection), one thread per cell, in place.
template <int K, bool ADJ, typename T, bool VR = false>
__global__ __launch_bounds__(TBX* TBY) void k_vel(Fields f, GridDims g, Coef cf, LineDev sl,
                                                  TraceIO so, LineDev il, TraceIO io) {
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
  const Pml<C> pm{static_cast<const C*>(cf.pml), P, g.NZ};
  // velocity coefficient: one value for constant density, else (VR) the one
  // of each velocity's own half node
  const C cbx = VR ? static_cast<const C*>(cf.cbx)[g.origin + o] : C(cf.cb);
  const C cbz = VR ? static_cast<const C*>(cf.cbz)[g.origin + o] : C(cf.cb);

  if (so.n >= 0 && I == sl.row0 && J >= sl.col0 && J < sl.col0 + sl.ntr) {
    const C val = C(sl.w0) * ldc<C>(p + o) + C(sl.w1) * ldc<C>(p + (long long)sl.row1 * P + J);
    line_out<C, V>(sl, so, J, shot, val);
  }

  C sx = C(0);
  bool split_x = false;
  if constexpr (ADJ) split_x = I < g.L || I >= g.NZ - g.L || J < g.L + K || J >= g.NX - g.L - K;
  if (!split_x) {
#pragma unroll
    for (int m = 1; m <= K; ++m)
      sx = acc(sx, wst<K, C>(m - 1), ldc<C>(p + o + m), ldc<C>(p + o + 1 - m));
  } else {
    // transposed x-split pressure P~_x = P~_z + aux (aux is zero off the frame)
    const T* __restrict__ ax = static_cast<const T*>(f.aux) + base;
#pragma unroll
    for (int m = 1; m <= K; ++m)
      sx = acc(sx, wst<K, C>(m - 1), ldc<C>(p + o + m) + ldc<C>(ax + o + m),
               ldc<C>(p + o + 1 - m) + ldc<C>(ax + o + 1 - m));
  }
  stc(vx + o, upd_v<ADJ>(pm.axh(J), pm.bxh(J), cbx, ldc<C>(vx + o), sx, C(0)));

  C sz = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m)
    sz = acc(sz, wst<K, C>(m - 1), ldc<C>(p + o + (long long)m * P),
             ldc<C>(p + o + (long long)(1 - m) * P));
  const C src = line_src<C, V>(il, io, I, J, shot);
  stc(vz + o, upd_v<ADJ>(pm.azh(I), pm.bzh(I), cbz, ldc<C>(vz + o), sz, src));
}

template <int K, bool ADJ, typename T>
__global__ __launch_bounds__(TBX* TBY) void k_pres(Fields f, GridDims g, Coef cf, LineDev sl,
                                                   TraceIO so, LineDev il, TraceIO io) {
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
  const Pml<C> pm{static_cast<const C*>(cf.pml), P, g.NZ};

  if (so.n >= 0 && I == sl.row0 && J >= sl.col0 && J < sl.col0 + sl.ntr) {
    const C val =
        C(sl.w0) * ldc<C>(vz + o) + C(sl.w1) * ldc<C>(vz + (long long)sl.row1 * P + J);
    line_out<C, V>(sl, so, J, shot, val);
  }

  C dx = C(0), dz = C(0);
#pragma unroll
  for (int m = 1; m <= K; ++m) {
    dx = acc(dx, wst<K, C>(m - 1), ldc<C>(vx + o + m - 1), ldc<C>(vx + o - m));
    dz = acc(dz, wst<K, C>(m - 1), ldc<C>(vz + o + (long long)(m - 1) * P),
             ldc<C>(vz + o - (long long)m * P));
  }
  const C src = line_src<C, V>(il, io, I, J, shot);
  const C ck = static_cast<const C*>(cf.ck)[g.origin + o];
  const C pc = ldc<C>(p + o);
  const bool frame = I < g.L || I >= g.NZ - g.L || J < g.L || J >= g.NX - g.L;
  C pn;
  if (!frame) {
    pn = upd_p<ADJ>(ck, pc, dx, dz, src);
  } else {
    T* __restrict__ au = static_cast<T*>(f.aux) + base;
    C an;
    pn = upd_p_frame<ADJ>(ck, pc, ldc<C>(au + o), dx, dz, src, pm.axn(J), pm.bxn(J), pm.azn(I),
                          pm.bzn(I), &an);
    stc(au + o, an);
  }
  stc(p + o, pn);
}

// ---------------------------------------------------------------------------
// Fused time step: one launch advances (p, v) by dt on a TX x TZ output tile
// (all shots in one grid).
//
// Every global load of a tile (p^n with a halo, the old velocities, ck, the
// frame auxiliaries; on general tiles also the layer factors, line trace
// values and field scales) is issued up front into registers, before the
// first wait, so that a tile pays one memory round trip.  Then p^n over
// the tile plus R = 2K-1 rows and 8 columns is staged in LDS; v^{n+1/2} is
// computed for the tile and the halo the pressure stencil needs (v_x on the
// tile rows over columns x0-4 .. x1+3, v_z on the tile columns over rows
// z0-K .. z1+K-2), the owned part is stored and the rest kept in LDS; last,
// p^{n+1} on the tile.  Each thread handles groups of 4 adjacent cells with
// 128-bit accesses.  Fields are double-buffered (in -> out), so neighbouring
// tiles never see a half-updated step.  Values outside the grid are zero
// (zero ghost cells around every field, rows outside [0, NZ) skipped).
//
// Tiles are ordered so that each XCD receives a contiguous band of tiles
// (workgroups are dispatched round-robin over the 8 XCDs), which keeps halo
// re-reads inside one L2.  A tile-loop form (k_step with LOOP = true) lets
// each workgroup take several interior tiles in turn, loading the next
// while computing the current one.
constexpr int TX = 64;
constexpr int HXS = 8;  // staged x halo (>= 2K - 1, multiple of 4)
// padding (floats) added to the LDS row pitch of the staged pressure, v_x
// and v_z tiles (multiples of 4: rows stay 16-byte aligned)
constexpr int LDS_PAD_P = 0, LDS_PAD_X = 0, LDS_PAD_Z = 0;

// threads of a fused-step workgroup: 256 for 64 x 8 and 64 x 16 tiles, 512
// for 64 x 32 (each thread owns the same 1 x 4 cells at every height)
constexpr int step_threads(int tz) { return tz == 32 ? 512 : 256; }

// waves per SIMD the fused step's register budget is set for: 6 (80 VGPRs)
// for one tile per workgroup, 4 (128) for the tile loop and for density
// arrays (velocity coefficients in registers), 2 (256) for FP64 values,
// which spill at 128
template <bool LOOP, bool VR, typename C>
constexpr int step_waves() { return sizeof(C) == 8 ? 2 : ((LOOP || VR) ? 4 : 6); }

// shape of the fused step's TX x TZ tile and of what it stages
template <int K, int TZ>
struct TileShape {
  static constexpr int NT = step_threads(TZ);
  static constexpr int R = 2 * K - 1;
  static constexpr int WP = TX + 2 * HXS;     // staged p columns: x0-8 .. x1+7
  static constexpr int GP = WP / 4;
  static constexpr int HP = TZ + 2 * R;       // staged p rows: z0-R .. z1+R-1
  static constexpr int GVX = TX / 4 + 2;      // v_x groups: x0-4 .. x1+3
  static constexpr int WVX = 4 * GVX;
  static constexpr int HVZ = TZ + 2 * K - 1;  // v_z rows: z0-K .. z1+K-2
  static constexpr int GT = TX / 4;           // groups per tile row
  // LDS pitches
  static constexpr int SPP = WP + LDS_PAD_P, SPX = WVX + LDS_PAD_X, SPZ = TX + LDS_PAD_Z;
  // 4-cell tasks per thread of each phase
  static constexpr int NQP = (HP * GP + NT - 1) / NT;
  static constexpr int NQX = (TZ * GVX + NT - 1) / NT;
  static constexpr int NQZ = (HVZ * GT + NT - 1) / NT;
  static constexpr int NQT = (TZ * GT + NT - 1) / NT;
  static constexpr int NQA = (TZ * GP + NT - 1) / NT;
  // general tiles' staged layer factors (offsets into sF, see step_general)
  static constexpr int FXH = 0, FXN = 2 * WVX, FZH = FXN + 2 * TX, FZN = FZH + 2 * HVZ;
  static constexpr int NF = FZN + 2 * TZ;
};

// an interior tile's loads, held in registers from their issue to the
// tile's compute phases
template <int K, int TZ, typename C, bool VR = false>
struct InteriorRegs {
  using S = TileShape<K, TZ>;
  C rp[S::NQP][4], rvx[S::NQX][4], rvz[S::NQZ][4], rck[S::NQT][4];
  // variable density: the velocity coefficients at the v_x and v_z cells
  C rbx[VR ? S::NQX : 1][4], rbz[VR ? S::NQZ : 1][4];
};

// no row of the line is active in rows [lo, hi)
__device__ __forceinline__ bool line_clear(const LineDev& l, const TraceIO& io, int lo, int hi) {
  return io.n < 0 || ((l.row0 < lo || l.row0 >= hi) && (l.row1 < lo || l.row1 >= hi));
}

// A tile is interior when everything it computes (v_x on columns x0-4 ..
// x1+3, v_z on rows z0-K .. z1+K-2, p on the tile) and everything it stages
// lies inside the absorbing frame's inner edge, where the layer factors a
// and b are exactly 1 at nodes and half nodes and the pressure is not split,
// and no line is sampled or injected in its rows.  Interior tiles take a
// path without per-cell tests; it evaluates the same expressions as the
// general path with a = b = 1 and zero sources, so results are bitwise
// equal.
// the absorbing-frame part of the test, and the rows a line must avoid
__host__ __device__ __forceinline__ bool interior_box(int K, int tz, int L, int NZ, int NX,
                                                      int x0, int z0) {
  const int R = 2 * K - 1;
  return z0 - R >= L && z0 + tz + R <= NZ - L - 1 && x0 - HXS >= L && x0 + TX + HXS <= NX - L - 1;
}
__host__ __device__ __forceinline__ int interior_rows_lo(int K, int z0) { return z0 - (2 * K - 1); }
__host__ __device__ __forceinline__ int interior_rows_hi(int K, int tz, int z0) {
  return z0 + tz + 2 * K - 1;
}

template <int K, int TZ>
__device__ __forceinline__ bool interior_tile(const StepArgs& a, int x0, int z0) {
  const int lo = interior_rows_lo(K, z0), hi = interior_rows_hi(K, TZ, z0);
  return interior_box(K, TZ, a.g.L, a.g.NZ, a.g.NX, x0, z0) && line_clear(a.vsl, a.vs, lo, hi) &&
         line_clear(a.vil, a.vi, lo, hi) && line_clear(a.psl, a.ps, lo, hi) &&
         line_clear(a.pil, a.pi, lo, hi);
}

// The step-history group (GradRows layout) of cells (I, J .. J+3), J a
// multiple of 4, of one shot: the residual of the pressure update is stored
// there by forward launches that carry a history pointer.
template <typename T>
__device__ __forceinline__ T* hist_group(const StepArgs& a, int shot, int I, int J) {
  const int L = a.g.L, nz = a.g.NZ - 2 * L, nx = a.g.NX - 2 * L;
  const GradRows gr(L, nx);
  return static_cast<T*>(a.hist) + ((long long)shot * nz + (I - L)) * gr.width() + (J - 4 * gr.g0);
}

// An interior tile's global loads (p^n with its halo, the old velocities,
// ck), issued into registers.
template <int K, typename T, int TZ, typename C, bool VR = false>
__device__ __forceinline__ void interior_load(const StepArgs& a, long long base, int x0, int z0,
                                              InteriorRegs<K, TZ, C, VR>& r) {
  using S = TileShape<K, TZ>;
  constexpr int NT = S::NT, R = S::R, GP = S::GP, HP = S::HP, GVX = S::GVX, HVZ = S::HVZ;
  constexpr int GT = S::GT, NQP = S::NQP, NQX = S::NQX, NQZ = S::NQZ, NQT = S::NQT;
  const int P = a.g.pitch;
  const int tid = threadIdx.x;
  const long long o0 = base + (long long)z0 * P + x0;  // element (z0, x0) of this shot
  const T* pA = static_cast<const T*>(a.in.p) + (o0 - (long long)R * P - HXS);
  const T* vxA = static_cast<const T*>(a.in.vx) + (o0 - 4);
  const T* vzA = static_cast<const T*>(a.in.vz) + (o0 - (long long)K * P);
  const C* ckA = static_cast<const C*>(a.c.ck) + (a.g.origin + (long long)z0 * P + x0);
  // (coefficient arrays have no shot stride: element (I, J) at origin + I P + J)
  const C* bxA = VR ? static_cast<const C*>(a.c.cbx) + (a.g.origin + (long long)z0 * P + x0 - 4)
                    : nullptr;
  const C* bzA = VR ? static_cast<const C*>(a.c.cbz) +
                          (a.g.origin + (long long)(z0 - K) * P + x0)
                    : nullptr;
#pragma unroll
  for (int k = 0; k < NQP; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < HP * GP || q < HP * GP) {
      const int rr = q / GP, g = q - rr * GP;
      ld4(r.rp[k], at(pA, rr * P + 4 * g));
    }
  }
#pragma unroll
  for (int k = 0; k < NQX; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < TZ * GVX || q < TZ * GVX) {
      const int rr = q / GVX, g = q - rr * GVX;
      ld4(r.rvx[k], at(vxA, rr * P + 4 * g));
      if constexpr (VR) ld4(r.rbx[k], at(bxA, rr * P + 4 * g));
    }
  }
#pragma unroll
  for (int k = 0; k < NQZ; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < HVZ * GT || q < HVZ * GT) {
      ld4(r.rvz[k], at(vzA, (q >> 4) * P + 4 * (q & 15)));
      if constexpr (VR) ld4(r.rbz[k], at(bzA, (q >> 4) * P + 4 * (q & 15)));
    }
  }
#pragma unroll
  for (int k = 0; k < NQT; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < TZ * GT || q < TZ * GT) ld4(r.rck[k], at(ckA, (q >> 4) * P + 4 * (q & 15)));
  }
}

// An interior tile's compute phases from its loaded registers: stage p^n,
// then (after the barrier, where after_stage() may issue the next tile's
// loads) v^{n+1/2} and p^{n+1}.  HIST: also store the residual of the
// pressure update (interior tiles hold physical cells only and no line).
template <int K, bool ADJ, typename T, int TZ, typename C, bool HIST, typename F,
          bool VR = false>
__device__ __forceinline__ void interior_compute(const StepArgs& a, int shot, long long base,
                                                 int x0, int z0,
                                                 const InteriorRegs<K, TZ, C, VR>& r,
                                                 C* __restrict__ sP, C* __restrict__ sVX,
                                                 C* __restrict__ sVZ, F&& after_stage) {
  using S = TileShape<K, TZ>;
  constexpr int NT = S::NT, R = S::R, GP = S::GP, HP = S::HP, GVX = S::GVX, HVZ = S::HVZ;
  constexpr int GT = S::GT, SPP = S::SPP, SPX = S::SPX, SPZ = S::SPZ;
  constexpr int NQP = S::NQP, NQX = S::NQX, NQZ = S::NQZ, NQT = S::NQT;
  const int P = a.g.pitch;
  const int tid = threadIdx.x;
  const long long o0 = base + (long long)z0 * P + x0;  // element (z0, x0) of this shot
  T* pB = static_cast<T*>(a.out.p) + o0;
  T* vxB = static_cast<T*>(a.out.vx) + (o0 - 4);
  T* vzB = static_cast<T*>(a.out.vz) + (o0 - (long long)K * P);
  const C cb = C(a.c.cb);
  const C one = C(1), zero = C(0);
  const auto& rvx = r.rvx;
  const auto& rvz = r.rvz;
  const auto& rck = r.rck;

  // ---- stage p^n -------------------------------------------------------------
#pragma unroll
  for (int k = 0; k < NQP; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < HP * GP || q < HP * GP) { const int rr = q / GP, g = q - rr * GP; st4(sP + rr * SPP + 4 * g, r.rp[k]); }
  }
  __syncthreads();
  after_stage();

  // ---- v_x on the tile rows, columns x0-4 .. x1+3 ------------------------------
#pragma unroll
  for (int k = 0; k < NQX; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < TZ * GVX || q < TZ * GVX) {
      const int rr = q / GVX, g = q - rr * GVX;
      const C* row = sP + (rr + R) * SPP + 4 * g;
      C w[12];
      ld4(*reinterpret_cast<C(*)[4]>(w), row);
      ld4(*reinterpret_cast<C(*)[4]>(w + 4), row + 4);
      ld4(*reinterpret_cast<C(*)[4]>(w + 8), row + 8);
      C val[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        C sx = zero;
#pragma unroll
        for (int m = 1; m <= K; ++m) sx = acc(sx, wst<K, C>(m - 1), w[e + 4 + m], w[e + 5 - m]);
        const C cbe = VR ? r.rbx[k][e] : cb;
        val[e] = rnd<T>(upd_v<ADJ>(one, one, cbe, rvx[k][e], sx, zero));
      }
      if (g >= 1 && g <= GT) st4(at(vxB, rr * P + 4 * g), val);
      st4(sVX + rr * SPX + 4 * g, val);
    }
  }
  // ---- v_z on the tile columns, rows z0-K .. z1+K-2 ----------------------------
#pragma unroll
  for (int k = 0; k < NQZ; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < HVZ * GT || q < HVZ * GT) {
      const int rr = q >> 4, g = q & 15;
      const C* col = sP + (rr - K + R) * SPP + 4 * g + HXS;
      C sz[4] = {zero, zero, zero, zero};
#pragma unroll
      for (int m = 1; m <= K; ++m) {
        C hi[4], lo[4];
        ld4(hi, col + m * SPP);
        ld4(lo, col + (1 - m) * SPP);
#pragma unroll
        for (int e = 0; e < 4; ++e) sz[e] = acc(sz[e], wst<K, C>(m - 1), hi[e], lo[e]);
      }
      C val[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const C cbe = VR ? r.rbz[k][e] : cb;
        val[e] = rnd<T>(upd_v<ADJ>(one, one, cbe, rvz[k][e], sz[e], zero));
      }
      if (rr >= K && rr < K + TZ) st4(at(vzB, rr * P + 4 * g), val);
      st4(sVZ + rr * SPZ + 4 * g, val);
    }
  }
  __syncthreads();

  // ---- p^{n+1} on the tile -------------------------------------------------------
#pragma unroll
  for (int k = 0; k < NQT; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < TZ * GT || q < TZ * GT) {
      const int rr = q >> 4, g = q & 15;
      C w[12];
      const C* vrow = sVX + rr * SPX + 4 * g;
      ld4(*reinterpret_cast<C(*)[4]>(w), vrow);
      ld4(*reinterpret_cast<C(*)[4]>(w + 4), vrow + 4);
      ld4(*reinterpret_cast<C(*)[4]>(w + 8), vrow + 8);
      C dx[4] = {zero, zero, zero, zero}, dz[4] = {zero, zero, zero, zero};
#pragma unroll
      for (int m = 1; m <= K; ++m) {
        C hi[4], lo[4];
        ld4(hi, sVZ + (rr + K + m - 1) * SPZ + 4 * g);
        ld4(lo, sVZ + (rr + K - m) * SPZ + 4 * g);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          dx[e] = acc(dx[e], wst<K, C>(m - 1), w[e + m + 3], w[e + 4 - m]);
          dz[e] = acc(dz[e], wst<K, C>(m - 1), hi[e], lo[e]);
        }
      }
      C pc[4], pn[4];
      ld4(pc, sP + (rr + R) * SPP + 4 * g + HXS);
#pragma unroll
      for (int e = 0; e < 4; ++e) pn[e] = upd_p<ADJ>(rck[k][e], pc[e], dx[e], dz[e], zero);
      st4(at(pB, rr * P + 4 * g), pn);
      if constexpr (HIST) {
        C rs[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) rs[e] = zero - (dx[e] + dz[e]);
        st4(hist_group<T>(a, shot, z0 + rr, x0 + 4 * g), rs);
      }
    }
  }
}

// A general tile (absorbing frame, lines, grid edges), loads included.
template <int K, bool ADJ, typename T, int TZ, typename C, bool HIST, bool VR = false>
__device__ __forceinline__ void step_general(const StepArgs& a, int shot, int x0, int z0,
                                             C* __restrict__ sP, C* __restrict__ sPX,
                                             C* __restrict__ sVX, C* __restrict__ sVZ,
                                             C* __restrict__ sF, C* __restrict__ sL) {
  using V = typename Tr<T>::V;
  using S = TileShape<K, TZ>;
  constexpr int NT = S::NT, R = S::R, GP = S::GP, HP = S::HP, GVX = S::GVX, WVX = S::WVX;
  constexpr int HVZ = S::HVZ, GT = S::GT, SPP = S::SPP, SPX = S::SPX, SPZ = S::SPZ;
  constexpr int NQP = S::NQP, NQX = S::NQX, NQZ = S::NQZ, NQT = S::NQT, NQA = S::NQA;
  constexpr int FXH = S::FXH, FXN = S::FXN, FZH = S::FZH, FZN = S::FZN;
  const int x1 = x0 + TX, z1 = z0 + TZ;
  const int NX = a.g.NX, NZ = a.g.NZ, P = a.g.pitch, L = a.g.L;
  const long long base = a.g.origin + (long long)shot * a.g.field_stride;
  // ---- general tiles: absorbing frame, lines, grid edges -----------------
  // Same expressions as the interior path, with the layer factors, the
  // frame split and the line terms, and with tile-uniform tests selecting
  // the per-cell work: columns or rows outside the grid hold zero, nothing
  // outside the grid is stored.  Ghost rows (GZ >= R) and columns (GX >= 8)
  // make every staged access of a tile above the last tile row land in
  // zeroed padding, so only that row predicates its loads.
  const C cb = C(a.c.cb);
  const int tid = threadIdx.x;
  const Pml<C> pm{static_cast<const C*>(a.c.pml), P, NZ};
  const bool frame_tile = (z0 < L) || (z1 > NZ - L) || (x0 < L) || (x1 > NX - L);
  const bool edge_x = x0 == 0 || x1 + 4 > NX;   // computed columns outside the grid
  const bool edge_z = z0 - K < 0 || z1 + K - 1 > NZ;  // computed rows outside the grid
  const bool rows_ok = z0 - R >= -GZ && z1 + R <= NZ + GZ;  // no load needs a row test
  const bool vil_here = !line_clear(a.vil, a.vi, z0 - K, z1 + K - 1);
  const bool pil_here = !line_clear(a.pil, a.pi, z0, z1);
  // the transposed x-stencil reads P~_x = P~_z + aux where the frame is near
  const bool use_px = ADJ && ((z0 < L) || (z1 > NZ - L) || (x0 - HXS < L) || (x1 + HXS > NX - L));
  static_assert(GZ >= R && GX >= HXS, "ghost padding narrower than the staged halo");

  const long long o0 = base + (long long)z0 * P + x0;  // element (z0, x0) of this shot
  const T* pA = static_cast<const T*>(a.in.p) + (o0 - (long long)R * P - HXS);
  const T* vxA = static_cast<const T*>(a.in.vx) + (o0 - 4);
  const T* vzA = static_cast<const T*>(a.in.vz) + (o0 - (long long)K * P);
  const T* auA = static_cast<const T*>(a.in.aux) + o0;
  const T* axA = static_cast<const T*>(a.in.aux) + (o0 - HXS);
  const C* ckA = static_cast<const C*>(a.c.ck) + (a.g.origin + (long long)z0 * P + x0);
  T* pB = static_cast<T*>(a.out.p) + o0;
  T* vxB = static_cast<T*>(a.out.vx) + (o0 - 4);
  T* vzB = static_cast<T*>(a.out.vz) + (o0 - (long long)K * P);
  T* auB = static_cast<T*>(a.out.aux) + o0;
  auto row_in = [&](int I) { return rows_ok || (I >= 0 && I < NZ); };

  // ---- loads ---------------------------------------------------------------
  C rp[NQP][4];
#pragma unroll
  for (int k = 0; k < NQP; ++k) {
    const int q = tid + NT * k;
#pragma unroll
    for (int e = 0; e < 4; ++e) rp[k][e] = C(0);
    if (NT * k + NT - 1 < HP * GP || q < HP * GP) {
      const int rr = q / GP, g = q - rr * GP;
      if (row_in(z0 - R + rr)) ld4(rp[k], at(pA, rr * P + 4 * g));
    }
  }
  // variable density: velocity coefficients at the v_x and v_z cells
  // (coefficient arrays have no shot stride; zero ghosts outside the grid)
  const C* bxA = VR ? static_cast<const C*>(a.c.cbx) + (a.g.origin + (long long)z0 * P + x0 - 4)
                    : nullptr;
  const C* bzA = VR ? static_cast<const C*>(a.c.cbz) +
                          (a.g.origin + (long long)(z0 - K) * P + x0)
                    : nullptr;
  C rvx[NQX][4], rbx[VR ? NQX : 1][4];
#pragma unroll
  for (int k = 0; k < NQX; ++k) {
    const int q = tid + NT * k;
#pragma unroll
    for (int e = 0; e < 4; ++e) rvx[k][e] = C(0);
    if constexpr (VR) {
#pragma unroll
      for (int e = 0; e < 4; ++e) rbx[k][e] = C(0);
    }
    if (NT * k + NT - 1 < TZ * GVX || q < TZ * GVX) {
      const int rr = q / GVX, g = q - rr * GVX;
      if (row_in(z0 + rr)) {
        ld4(rvx[k], at(vxA, rr * P + 4 * g));
        if constexpr (VR) ld4(rbx[k], at(bxA, rr * P + 4 * g));
      }
    }
  }
  C rvz[NQZ][4], rbz[VR ? NQZ : 1][4];
#pragma unroll
  for (int k = 0; k < NQZ; ++k) {
    const int q = tid + NT * k;
#pragma unroll
    for (int e = 0; e < 4; ++e) rvz[k][e] = C(0);
    if constexpr (VR) {
#pragma unroll
      for (int e = 0; e < 4; ++e) rbz[k][e] = C(0);
    }
    if ((NT * k + NT - 1 < HVZ * GT || q < HVZ * GT) && row_in(z0 - K + (q >> 4))) {
      ld4(rvz[k], at(vzA, (q >> 4) * P + 4 * (q & 15)));
      if constexpr (VR) ld4(rbz[k], at(bzA, (q >> 4) * P + 4 * (q & 15)));
    }
  }
  C rck[NQT][4], rau[NQT][4];
#pragma unroll
  for (int k = 0; k < NQT; ++k) {
    const int q = tid + NT * k;
#pragma unroll
    for (int e = 0; e < 4; ++e) rck[k][e] = rau[k][e] = C(0);
    if ((NT * k + NT - 1 < TZ * GT || q < TZ * GT) && row_in(z0 + (q >> 4))) {
      const unsigned off = (q >> 4) * P + 4 * (q & 15);
      ld4(rck[k], at(ckA, off));
      if (frame_tile) ld4(rau[k], at(auA, off));
    }
  }
  C rax[ADJ ? NQA : 1][4];
  if constexpr (ADJ) {
#pragma unroll
    for (int k = 0; k < NQA; ++k) {
      const int q = tid + NT * k;
#pragma unroll
      for (int e = 0; e < 4; ++e) rax[k][e] = C(0);
      if (use_px && (NT * k + NT - 1 < TZ * GP || q < TZ * GP)) {
        const int rr = q / GP, g = q - rr * GP;
        if (row_in(z0 + rr)) ld4(rax[k], at(axA, rr * P + 4 * g));
      }
    }
  }
  // layer factors (the padded arrays hold 1 outside the grid): the x
  // factors as 128-bit groups, the z factors one per thread
  // factors, only in a direction in which the tile reaches the layer
  // (half nodes are 1 on [L, N-L-1), nodes on [L, N-L))
  // Their values are loaded into registers here, together with the fields
  // (one memory round trip for every load of the tile), and stored to LDS
  // with the staged p below.
  static_assert(NT >= 2 * GVX + 2 * GT + 2 * HVZ + 2 * TZ, "too few threads for the factors");
  const bool lay_x = x0 - 4 < L || x1 + 4 > NX - L - 1;
  const bool lay_z = z0 - K < L || z1 + K - 1 > NZ - L - 1;
  // One load per kind and thread, into registers of its own (loads of
  // different branches into the same registers would each wait for the
  // last): four x factors (a_h, b_h over the v_x groups, then a_n, b_n over
  // the tile's groups) or one z factor (a_h, b_h over the v_z rows, then
  // a_n, b_n over the tile's rows).
  C fx[4] = {C(1), C(1), C(1), C(1)};
  C fz = C(1);
  constexpr int NFX = 2 * GVX + 2 * GT, NFZ = 2 * HVZ + 2 * TZ;
  // (two independent tests, both values set before either load: written
  // inside the other branch, a default would wait for the load in flight)
  const bool fxt = tid < NFX, fzt = tid >= NFX && tid < NFX + NFZ;
  int fslot;  // sF slot of this thread's x group (fx) or z entry (fz)
  {
    const bool h = tid < 2 * GVX;
    const int j = h ? tid : tid - 2 * GVX;
    const int n = h ? GVX : GT;  // groups per factor
    const int which = (h ? 2 : 0) + (j < n ? 0 : 1);
    const int col = (h ? x0 - 4 : x0) + 4 * (j < n ? j : j - n);
    if (fxt && lay_x) ld4(fx, pm.xa(which, col));
    fslot = (h ? FXH : FXN) + 4 * j;
  }
  {
    const int i = tid - NFX;
    const bool h = i < 2 * HVZ;
    const int j = h ? i : i - 2 * HVZ;
    const int n = h ? HVZ : TZ;  // rows per factor
    const int which = (h ? 2 : 0) + (j < n ? 0 : 1);
    const int row = (h ? z0 - K : z0) + (j < n ? j : j - n);
    if (fzt && lay_z) fz = *pm.za(which, row);
    if (fzt) fslot = (h ? FZH : FZN) + j;
  }
  // line injections (0 off the line), with the arithmetic of line_src: the
  // trace value and the field scales are loaded here, the value formed
  // when it is stored
  const bool lthread = (vil_here || pil_here) && tid < 4 * TX;
  const int lj = tid >> 6, lc = tid & (TX - 1);  // 4 rows of TX values
  const LineDev& ll = lj < 2 ? a.vil : a.pil;
  const TraceIO& lio = lj < 2 ? a.vi : a.pi;
  const int lrow = (lj & 1) ? ll.row1 : ll.row0, lcol = x0 + lc;
  const bool lon = lthread && lio.n >= 0 && (lrow == ll.row0 || lrow == ll.row1) &&
                   lcol >= ll.col0 && lcol < ll.col0 + ll.ntr;
  C lraw = C(0), ldyn = C(1);
  if (lon) {
    lraw = C(*(static_cast<const V*>(lio.in) + shot * lio.shot_stride + (long long)lio.n * ll.ntr +
               (lcol - ll.col0)));
    ldyn = dyn_of<C>(lio, shot);
  }
  // field scales of the sampled lines
  const C dyn_vs = a.vs.n >= 0 ? dyn_of<C>(a.vs, shot) : C(1);
  const C dyn_ps = a.ps.n >= 0 ? dyn_of<C>(a.ps, shot) : C(1);

  // ---- stage p^n (and P~_x), the layer factors and the line values ---------
#pragma unroll
  for (int k = 0; k < NQP; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < HP * GP || q < HP * GP) { const int rr = q / GP, g = q - rr * GP; st4(sP + rr * SPP + 4 * g, rp[k]); }
  }
  if (fxt) st4(sF + fslot, fx);
  if (fzt) sF[fslot] = fz;
  if (lthread) {
    const C w = (lrow == ll.row0 ? C(ll.w0) : C(0)) + (lrow == ll.row1 ? C(ll.w1) : C(0));
    sL[tid] = lon ? w * (C(lio.scale) * lraw / ldyn) : C(0);
  }
  if constexpr (ADJ) {
    if (use_px) {
#pragma unroll
      for (int k = 0; k < NQA; ++k) {
        const int q = tid + NT * k;
        if (NT * k + NT - 1 < TZ * GP || q < TZ * GP) { const int rr = q / GP, g = q - rr * GP; st4(sPX + rr * SPP + 4 * g, rax[k]); }
      }
    }
  }
  __syncthreads();
  if constexpr (ADJ) {
    if (use_px) {
      // P~_x = P~_z + aux (tile row rr of sPX is row rr + R of sP)
#pragma unroll
      for (int k = 0; k < NQA; ++k) {
        const int q = tid + NT * k;
        if (NT * k + NT - 1 < TZ * GP || q < TZ * GP) {
          const int rr = q / GP, g = q - rr * GP;
          C pz[4], ax[4], sum[4];
          ld4(pz, sP + (rr + R) * SPP + 4 * g);
          ld4(ax, sPX + rr * SPP + 4 * g);
#pragma unroll
          for (int e = 0; e < 4; ++e) sum[e] = pz[e] + ax[e];
          st4(sPX + rr * SPP + 4 * g, sum);
        }
      }
      __syncthreads();
    }
  }

  // pressure-line sampling (p^n)
  if (a.vs.n >= 0 && a.vsl.row0 >= z0 && a.vsl.row0 < z1 && tid < TX) {
    const int J = x0 + tid;
    if (J >= a.vsl.col0 && J < a.vsl.col0 + a.vsl.ntr && J < NX) {
      const int r0 = a.vsl.row0 - z0 + R, r1 = a.vsl.row1 - z0 + R;
      const C val =
          C(a.vsl.w0) * sP[r0 * SPP + tid + HXS] + C(a.vsl.w1) * sP[r1 * SPP + tid + HXS];
      V* out = static_cast<V*>(a.vs.out) + shot * a.vs.shot_stride + (long long)a.vs.n * a.vsl.ntr +
               (J - a.vsl.col0);
      *out = V(C(a.vs.scale) * val * dyn_vs);  // the arithmetic of line_out
    }
  }

  // ---- v_x on the tile rows, columns x0-4 .. x1+3 ------------------------------
#pragma unroll
  for (int k = 0; k < NQX; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < TZ * GVX || q < TZ * GVX) {
      const int rr = q / GVX, g = q - rr * GVX;
      const int I = z0 + rr, J = x0 - 4 + 4 * g;
      const C* row = (ADJ && use_px) ? (sPX + rr * SPP + 4 * g) : (sP + (rr + R) * SPP + 4 * g);
      C w[12];  // staged p (transposed: P~_x) at columns J-4 .. J+7
      ld4(*reinterpret_cast<C(*)[4]>(w), row);
      ld4(*reinterpret_cast<C(*)[4]>(w + 4), row + 4);
      ld4(*reinterpret_cast<C(*)[4]>(w + 8), row + 8);
      C ax[4], bx[4];
      ld4(ax, sF + FXH + 4 * g);
      ld4(bx, sF + FXH + WVX + 4 * g);
      C val[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        C sx = C(0);
#pragma unroll
        for (int m = 1; m <= K; ++m) sx = acc(sx, wst<K, C>(m - 1), w[e + 4 + m], w[e + 5 - m]);
        const C cbe = VR ? rbx[k][e] : cb;
        val[e] = rnd<T>(upd_v<ADJ>(ax[e], bx[e], cbe, rvx[k][e], sx, C(0)));
        if (edge_x && (J + e < 0 || J + e >= NX)) val[e] = C(0);  // outside the grid
      }
      if (g >= 1 && g <= GT && I < NZ) {
        if (!edge_x || J + 3 < NX) {
          st4(at(vxB, rr * P + 4 * g), val);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (J + e < NX) stc(at(vxB, rr * P + 4 * g + e), val[e]);
        }
      }
      st4(sVX + rr * SPX + 4 * g, val);
    }
  }
  // ---- v_z on the tile columns, rows z0-K .. z1+K-2 ----------------------------
#pragma unroll
  for (int k = 0; k < NQZ; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < HVZ * GT || q < HVZ * GT) {
      const int rr = q >> 4, g = q & 15;
      const int I = z0 - K + rr, J = x0 + 4 * g;
      const C* col = sP + (rr - K + R) * SPP + 4 * g + HXS;
      C sz[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
      for (int m = 1; m <= K; ++m) {
        C hi[4], lo[4];
        ld4(hi, col + m * SPP);
        ld4(lo, col + (1 - m) * SPP);
#pragma unroll
        for (int e = 0; e < 4; ++e) sz[e] = acc(sz[e], wst<K, C>(m - 1), hi[e], lo[e]);
      }
      const C az = sF[FZH + rr], bz = sF[FZH + HVZ + rr];
      const bool row_ok = !edge_z || (I >= 0 && I < NZ);
      const C* lrow = !vil_here ? nullptr
                      : I == a.vil.row0 ? sL : (I == a.vil.row1 ? sL + TX : nullptr);
      C val[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const C src = lrow ? lrow[4 * g + e] : C(0);
        const C cbe = VR ? rbz[k][e] : cb;
        val[e] = rnd<T>(upd_v<ADJ>(az, bz, cbe, rvz[k][e], sz[e], src));
        if (!row_ok || (edge_x && J + e >= NX)) val[e] = C(0);  // outside the grid
      }
      if (rr >= K && rr < K + TZ && I < NZ) {
        if (!edge_x || J + 3 < NX) {
          st4(at(vzB, rr * P + 4 * g), val);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (J + e < NX) stc(at(vzB, rr * P + 4 * g + e), val[e]);
        }
      }
      st4(sVZ + rr * SPZ + 4 * g, val);
    }
  }
  __syncthreads();

  // v_z-line sampling (v^{n+1/2})
  if (a.ps.n >= 0 && a.psl.row0 >= z0 && a.psl.row0 < z1 && tid < TX) {
    const int J = x0 + tid;
    if (J >= a.psl.col0 && J < a.psl.col0 + a.psl.ntr && J < NX) {
      const int r0 = a.psl.row0 - z0 + K, r1 = a.psl.row1 - z0 + K;
      const C val = C(a.psl.w0) * sVZ[r0 * SPZ + tid] + C(a.psl.w1) * sVZ[r1 * SPZ + tid];
      V* out = static_cast<V*>(a.ps.out) + shot * a.ps.shot_stride + (long long)a.ps.n * a.psl.ntr +
               (J - a.psl.col0);
      *out = V(C(a.ps.scale) * val * dyn_ps);  // the arithmetic of line_out
    }
  }

  // ---- p^{n+1} on the tile -------------------------------------------------------
#pragma unroll
  for (int k = 0; k < NQT; ++k) {
    const int q = tid + NT * k;
    if (NT * k + NT - 1 < TZ * GT || q < TZ * GT) {
      const int rr = q >> 4, g = q & 15;
      const int I = z0 + rr, J = x0 + 4 * g;
      if (I >= NZ || J >= NX) continue;
      C w[12];  // v_x at columns J-4 .. J+7
      const C* vrow = sVX + rr * SPX + 4 * g;
      ld4(*reinterpret_cast<C(*)[4]>(w), vrow);
      ld4(*reinterpret_cast<C(*)[4]>(w + 4), vrow + 4);
      ld4(*reinterpret_cast<C(*)[4]>(w + 8), vrow + 8);
      C dx[4] = {C(0), C(0), C(0), C(0)}, dz[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
      for (int m = 1; m <= K; ++m) {
        C hi[4], lo[4];
        ld4(hi, sVZ + (rr + K + m - 1) * SPZ + 4 * g);
        ld4(lo, sVZ + (rr + K - m) * SPZ + 4 * g);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          dx[e] = acc(dx[e], wst<K, C>(m - 1), w[e + m + 3], w[e + 4 - m]);
          dz[e] = acc(dz[e], wst<K, C>(m - 1), hi[e], lo[e]);
        }
      }
      C pc[4], pn[4], an[4];
      ld4(pc, sP + (rr + R) * SPP + 4 * g + HXS);
      const C* lrow = !pil_here ? nullptr
                      : I == a.pil.row0 ? sL + 2 * TX : (I == a.pil.row1 ? sL + 3 * TX : nullptr);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int Je = J + e;
        const C src = lrow ? lrow[4 * g + e] : C(0);
        const bool frame = frame_tile && (I < L || I >= NZ - L || Je < L || Je >= NX - L);
        an[e] = rau[k][e];
        if (!frame) {
          pn[e] = upd_p<ADJ>(rck[k][e], pc[e], dx[e], dz[e], src);
        } else {
          pn[e] = upd_p_frame<ADJ>(rck[k][e], pc[e], rau[k][e], dx[e], dz[e], src,
                                   sF[FXN + 4 * g + e], sF[FXN + TX + 4 * g + e],
                                   sF[FZN + rr], sF[FZN + TZ + rr], &an[e]);
        }
      }
      if constexpr (HIST) {
        // physical rows; groups that meet the physical columns (others zero)
        if (I >= L && I < NZ - L && J + 3 >= L && J < NX - L) {
          C rs[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int Je = J + e;
            const C src = lrow ? lrow[4 * g + e] : C(0);
            rs[e] = (Je >= L && Je < NX - L) ? src - (dx[e] + dz[e]) : C(0);
          }
          st4(hist_group<T>(a, shot, I, J), rs);
        }
      }
      const unsigned off = rr * P + 4 * g;
      if (!edge_x || J + 3 < NX) {
        st4(at(pB, off), pn);
        if (frame_tile) st4(at(auB, off), an);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (J + e < NX) {
            stc(at(pB, off + e), pn[e]);
            if (frame_tile) stc(at(auB, off + e), an[e]);
          }
        }
      }
    }
  }
}

// XCD-aware tile order: logical index Lg -> tile.  Workgroups are
// dispatched round-robin over the 8 XCDs and workgroup b takes logical
// indices congruent to b mod 8, so each XCD receives a contiguous band of
// tiles, which keeps halo re-reads inside one L2.
__device__ __forceinline__ int xcd_tile(int Lg, int ntiles) {
  const int full = ntiles >> 3, rem = ntiles & 7, xcd = Lg & 7;
  return xcd * full + (xcd < rem ? xcd : rem) + (Lg >> 3);
}

// Fused one-step kernel.
//   LOOP = false: one tile per workgroup, the grid covers every tile.
//   LOOP = true (tile lists in a.tiles): the first nshots * ngen workgroups
//   take one general tile each; the others, a multiple of 8 no larger than
//   what the device holds at once, loop over the interior tiles (logical
//   indices b, b + G, b + 2G, ...) and issue the next tile's loads right
//   after staging the current one, so that its memory traffic overlaps the
//   current tile's compute instead of every workgroup loading, computing and
//   storing in step.  (General tiles stay outside the loop: inside it, their
//   long path raises register use past the point of spilling.)
template <int K, bool ADJ, typename T, int TZ, bool LOOP, bool HIST = false, bool VR = false>
__global__ __launch_bounds__(step_threads(TZ), (step_waves<LOOP, VR, typename Tr<T>::C>())) void k_step(StepArgs a) {
  static_assert(!(VR && (LOOP || HIST)), "variable density: one tile per workgroup, no history");
  using C = typename Tr<T>::C;
  using S = TileShape<K, TZ>;
  static_assert(2 * K - 1 <= HXS && K <= 4, "halo wider than the staged columns");
  __shared__ __align__(16) C sP[S::HP * S::SPP];
  __shared__ __align__(16) C sPX[ADJ ? TZ * S::SPP : 4];
  __shared__ __align__(16) C sVX[TZ * S::SPX];
  __shared__ __align__(16) C sVZ[S::HVZ * S::SPZ];
  // general tiles: layer factors and line injections, staged with the
  // loads so that no global access waits inside the compute phases
  //   sF: a_h, b_h over the v_x columns x0-4 .. x1+3; a_n, b_n over the
  //       tile's columns; a_h, b_h over the v_z rows; a_n, b_n over the
  //       tile's rows
  //   sL: injected values of the v_z line (rows row0, row1) and of the
  //       pressure line (rows row0, row1) over the tile's columns
  __shared__ __align__(16) C sF[S::NF];
  __shared__ __align__(16) C sL[4 * TX];

  auto base_of = [&](int shot) { return a.g.origin + (long long)shot * a.g.field_stride; };
  if constexpr (!LOOP) {
    const int per_shot = a.ntx * a.ntz;
    const int t = xcd_tile(blockIdx.x, per_shot * a.nshots);
    const int shot = t / per_shot;
    const int tt = t - shot * per_shot;
    const int tzi = tt / a.ntx;
    const int x0 = (tt - tzi * a.ntx) * TX, z0 = tzi * TZ;
    if (interior_tile<K, TZ>(a, x0, z0)) {
      InteriorRegs<K, TZ, C, VR> r;
      interior_load<K, T, TZ, C, VR>(a, base_of(shot), x0, z0, r);
      interior_compute<K, ADJ, T, TZ, C, HIST>(a, shot, base_of(shot), x0, z0, r, sP, sVX, sVZ,
                                               [] {});
    } else {
      step_general<K, ADJ, T, TZ, C, HIST, VR>(a, shot, x0, z0, sP, sPX, sVX, sVZ, sF, sL);
    }
  } else {
    const int ngen_all = a.nshots * a.ngen, nint_all = a.nshots * a.nint;
    if ((int)blockIdx.x < ngen_all) {
      const int idx = xcd_tile(blockIdx.x, ngen_all);
      const int shot = idx / a.ngen;
      const int e = __builtin_amdgcn_readfirstlane(idx - shot * a.ngen);
      const int tt = ((const __attribute__((address_space(4))) int*)a.tiles)[e];  // scalar load
      const int tzi = tt / a.ntx;
      step_general<K, ADJ, T, TZ, C, HIST>(a, shot, (tt - tzi * a.ntx) * TX, tzi * TZ, sP, sPX,
                                           sVX, sVZ, sF, sL);
      return;
    }
    // interior tiles: logical index Li -> (shot, x0, z0); the list entry is
    // read as constant memory with a uniform index, i.e. by a scalar load (a
    // vector load here would be waited for right away, and that wait would
    // also wait for every load in flight)
    auto locate = [&](int Li, int& shot, int& x0, int& z0) {
      const int idx = xcd_tile(Li, nint_all);
      shot = idx / a.nint;
      const int e = __builtin_amdgcn_readfirstlane(a.ngen + idx - shot * a.nint);
      const int tt = ((const __attribute__((address_space(4))) int*)a.tiles)[e];
      const int tzi = tt / a.ntx;
      x0 = (tt - tzi * a.ntx) * TX;
      z0 = tzi * TZ;
    };
    const int G = (int)gridDim.x - ngen_all;
    int Li = (int)blockIdx.x - ngen_all, shot, x0, z0;
    locate(Li, shot, x0, z0);
    // two register sets: the current tile's loads (staged, then read by its
    // compute phases) and the next tile's, issued once the current tile is
    // staged and in flight through its compute, then copied at the end of
    // the iteration.  (The compiler waits on part of the next tile's loads
    // inside the compute phases.  A form that avoids those waits, by
    // waiting for the first tile's loads before the loop and copying at the
    // top of it, measured 4 % slower on a c2 step and is not used.)
    InteriorRegs<K, TZ, C> cur, nxt;
    interior_load<K, T, TZ, C>(a, base_of(shot), x0, z0, cur);
    for (;;) {
      const int Ln = Li + G;
      const bool more = Ln < nint_all;
      int shotn = 0, x0n = 0, z0n = 0;
      if (more) locate(Ln, shotn, x0n, z0n);
      interior_compute<K, ADJ, T, TZ, C, HIST>(a, shot, base_of(shot), x0, z0, cur, sP, sVX, sVZ,
                                               [&] {
        if (more) interior_load<K, T, TZ, C>(a, base_of(shotn), x0n, z0n, nxt);
      });
      if (!more) break;
      __syncthreads();  // every read of this tile's LDS precedes the next staging
      cur = nxt;
      Li = Ln;
      shot = shotn;
      x0 = x0n;
      z0 = z0n;
    }
  }
}

// Several grids advanced by one time step in one launch (a heterogeneous
// batch): problem p takes blocks [b.pre[p], b.pre[p+1]) -- its tile count
// rounded up to a multiple of 8, so that the XCD-aware tile order of the
// one-grid kernel carries over -- and reads its step arguments from the
// launch's own argument block.  Each tile runs the one-tile-per-workgroup
// path of k_step (no history), so every grid's result is bitwise that of
// its own launch.
template <int K, bool ADJ, typename T, int TZ, bool VR>
__global__ __launch_bounds__(step_threads(TZ), (step_waves<false, VR, typename Tr<T>::C>())) void k_step_batch(BatchStep b) {
  using C = typename Tr<T>::C;
  using S = TileShape<K, TZ>;
  __shared__ __align__(16) C sP[S::HP * S::SPP];
  __shared__ __align__(16) C sPX[ADJ ? TZ * S::SPP : 4];
  __shared__ __align__(16) C sVX[TZ * S::SPX];
  __shared__ __align__(16) C sVZ[S::HVZ * S::SPZ];
  __shared__ __align__(16) C sF[S::NF];
  __shared__ __align__(16) C sL[4 * TX];
  int p = 0;
  for (int i = 1; i < b.n; ++i)
    if ((int)blockIdx.x >= b.pre[i]) p = i;
  const StepArgs& a = b.a[p];
  const int per_shot = a.ntx * a.ntz, ntiles = per_shot * a.nshots;
  const int t = xcd_tile((int)blockIdx.x - b.pre[p], b.pre[p + 1] - b.pre[p]);
  if (t >= ntiles) return;  // padding block
  const int shot = t / per_shot;
  const int tt = t - shot * per_shot;
  const int tzi = tt / a.ntx;
  const int x0 = (tt - tzi * a.ntx) * TX, z0 = tzi * TZ;
  const long long base = a.g.origin + (long long)shot * a.g.field_stride;
  if (interior_tile<K, TZ>(a, x0, z0)) {
    InteriorRegs<K, TZ, C, VR> r;
    interior_load<K, T, TZ, C, VR>(a, base, x0, z0, r);
    interior_compute<K, ADJ, T, TZ, C, false>(a, shot, base, x0, z0, r, sP, sVX, sVZ, [] {});
  } else {
    step_general<K, ADJ, T, TZ, C, false, VR>(a, shot, x0, z0, sP, sPX, sVX, sVZ, sF, sL);
  }
}

// ---------------------------------------------------------------------------
// line sampling after the last forward step, and a fill kernel

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
  line_out<C, V>(sl, so, J, shot, val);
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
  if (c.cbx)
    hipLaunchKernelGGL((k_vel<K, ADJ, T, true>), grid, dim3(TBX, TBY), 0, s, f, g, c, sl, so, il,
                       io);
  else
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
// Compute units of device dev and workgroups of `threads` threads of
// `kernel` that one of them holds at once, queried once per kernel and
// device and then cached (launches in eager mode would otherwise query at
// every step).
static hipError_t resident_blocks(const void* kernel, int threads, int dev, int* cus, int* occ) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, std::pair<int, int>> cache;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({kernel, dev});
  if (it == cache.end()) {
    int c = 0, o = 0;
    hipError_t e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kernel, threads, 0);
    if (e != hipSuccess) return e;
    it = cache.emplace(std::make_pair(kernel, dev), std::make_pair(c, o)).first;
  }
  *cus = it->second.first;
  *occ = it->second.second;
  return hipSuccess;
}

#define SSX_HIP_RET(x)                 \
  do {                                 \
    const hipError_t e_ = (x);         \
    if (e_ != hipSuccess) return e_;   \
  } while (0)

template <int K, bool ADJ, typename T>
static hipError_t step_t(int tz, int loop, const StepArgs& a, hipStream_t s) {
  const int ntiles = a.ntx * a.ntz * a.nshots;
  if (ntiles <= 0) return hipSuccess;
  // one tile per workgroup; or (loop) one workgroup per general tile plus
  // a looping set, a multiple of 8 no larger than what the device holds
  auto go = [&](auto kernel, int threads) -> hipError_t {
    int nb = ntiles;
    if (loop) {
      if (!a.tiles || a.ngen + a.nint != a.ntx * a.ntz) return hipErrorInvalidValue;
      int dev = 0, cus = 0, occ = 0;
      SSX_HIP_RET(hipGetDevice(&dev));
      SSX_HIP_RET(resident_blocks(reinterpret_cast<const void*>(kernel), threads, dev, &cus, &occ));
      int cap = std::max(8, cus * std::max(occ, 1) / 8 * 8);
      if (loop >= 8) cap = std::min(cap, loop / 8 * 8);
      nb = a.nshots * a.ngen + std::min(a.nshots * a.nint, cap);
    }
    hipLaunchKernelGGL(kernel, dim3(nb), dim3(threads), 0, s, a);
    return hipGetLastError();
  };
  if (a.c.cbx) {
    // variable density: one tile per workgroup, no step history
    if (loop || a.hist) return hipErrorInvalidValue;
    switch (tz) {
      case 8: return go(k_step<K, ADJ, T, 8, false, false, true>, step_threads(8));
      case 16: return go(k_step<K, ADJ, T, 16, false, false, true>, step_threads(16));
      case 32:
        if constexpr (sizeof(T) < 8)
          return go(k_step<K, ADJ, T, 32, false, false, true>, step_threads(32));
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
  }
  if (a.hist) {
    // the step history: forward steps with FP32 or FP64 fields only
    if constexpr (!ADJ && sizeof(T) >= 4) {
      switch (tz) {
        case 8:
          return loop ? go(k_step<K, ADJ, T, 8, true, true>, step_threads(8))
                      : go(k_step<K, ADJ, T, 8, false, true>, step_threads(8));
        case 16:
          return loop ? go(k_step<K, ADJ, T, 16, true, true>, step_threads(16))
                      : go(k_step<K, ADJ, T, 16, false, true>, step_threads(16));
        case 32:
          if constexpr (sizeof(T) < 8) {
            return loop ? go(k_step<K, ADJ, T, 32, true, true>, step_threads(32))
                        : go(k_step<K, ADJ, T, 32, false, true>, step_threads(32));
          }
          return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
      }
    }
    return hipErrorInvalidValue;
  }
  switch (tz) {
    case 8:
      return loop ? go(k_step<K, ADJ, T, 8, true>, step_threads(8))
                  : go(k_step<K, ADJ, T, 8, false>, step_threads(8));
    case 16:
      return loop ? go(k_step<K, ADJ, T, 16, true>, step_threads(16))
                  : go(k_step<K, ADJ, T, 16, false>, step_threads(16));
    case 32:
      if constexpr (sizeof(T) < 8) {
        return loop ? go(k_step<K, ADJ, T, 32, true>, step_threads(32))
                    : go(k_step<K, ADJ, T, 32, false>, step_threads(32));
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

#define SSX_DISPATCH(FN, ...)                                                        \
  do {                                                                               \
    const bool o8 = (order == 8);                                                    \
    switch (dt) {                                                                    \
      case Dt::F64:                                                                  \
        if (o8) return adj ? FN<4, true, double>(__VA_ARGS__) : FN<4, false, double>(__VA_ARGS__); \
        return adj ? FN<2, true, double>(__VA_ARGS__) : FN<2, false, double>(__VA_ARGS__);         \
      case Dt::F32:                                                                  \
        if (o8) return adj ? FN<4, true, float>(__VA_ARGS__) : FN<4, false, float>(__VA_ARGS__);   \
        return adj ? FN<2, true, float>(__VA_ARGS__) : FN<2, false, float>(__VA_ARGS__);           \
      case Dt::F16:                                                                  \
        if (o8) return adj ? FN<4, true, __half>(__VA_ARGS__) : FN<4, false, __half>(__VA_ARGS__); \
        return adj ? FN<2, true, __half>(__VA_ARGS__) : FN<2, false, __half>(__VA_ARGS__);         \
      case Dt::BF16:                                                                 \
        if (o8)                                                                      \
          return adj ? FN<4, true, __hip_bfloat16>(__VA_ARGS__)                     \
                     : FN<4, false, __hip_bfloat16>(__VA_ARGS__);                   \
        return adj ? FN<2, true, __hip_bfloat16>(__VA_ARGS__)                       \
                   : FN<2, false, __hip_bfloat16>(__VA_ARGS__);                     \
    }                                                                                \
    return hipErrorInvalidValue;                                                     \
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

void step_tile_lists(int order, int tz, const GridDims& g, const LineDev* const* lines,
                     int nlines, std::vector<int>* gen, std::vector<int>* inter) {
  const int K = order / 2;
  const int ntx = (g.NX + TX - 1) / TX, ntz = (g.NZ + tz - 1) / tz;
  gen->clear();
  inter->clear();
  for (int tzi = 0; tzi < ntz; ++tzi) {
    const int z0 = tzi * tz, lo = interior_rows_lo(K, z0), hi = interior_rows_hi(K, tz, z0);
    bool rows_ok = true;
    for (int i = 0; i < nlines; ++i) {
      const LineDev& l = *lines[i];
      if ((l.row0 >= lo && l.row0 < hi) || (l.row1 >= lo && l.row1 < hi)) rows_ok = false;
    }
    for (int txi = 0; txi < ntx; ++txi) {
      const bool in = rows_ok && interior_box(K, tz, g.L, g.NZ, g.NX, txi * TX, z0);
      (in ? inter : gen)->push_back(tzi * ntx + txi);
    }
  }
}

hipError_t launch_step(Dt dt, int order, bool adj, int tz, int loop, StepArgs a, hipStream_t s) {
  SSX_DISPATCH(step_t, tz, loop, a, s);
}

template <int K, bool ADJ, typename T>
static hipError_t step_batch_t(const BatchStep& b, bool vr, hipStream_t s) {
  if (b.n < 1 || b.n > BATCH_MAX || b.pre[0] != 0) return hipErrorInvalidValue;
  for (int i = 0; i < b.n; ++i) {
    const StepArgs& a = b.a[i];
    const int need = a.ntx * a.ntz * a.nshots;
    if ((a.c.cbx != nullptr) != vr || a.tiles || a.hist || b.pre[i + 1] - b.pre[i] < need ||
        (b.pre[i + 1] - b.pre[i]) % 8 != 0 || a.ntx != (a.g.NX + TX - 1) / TX ||
        a.ntz != (a.g.NZ + BATCH_TZ - 1) / BATCH_TZ)
      return hipErrorInvalidValue;
  }
  const dim3 grid(b.pre[b.n]), block(step_threads(BATCH_TZ));
  if (vr)
    hipLaunchKernelGGL((k_step_batch<K, ADJ, T, BATCH_TZ, true>), grid, block, 0, s, b);
  else
    hipLaunchKernelGGL((k_step_batch<K, ADJ, T, BATCH_TZ, false>), grid, block, 0, s, b);
  return hipGetLastError();
}

hipError_t launch_step_batch(Dt dt, int order, bool adj, bool vr, const BatchStep& b,
                             hipStream_t s) {
  SSX_DISPATCH(step_batch_t, b, vr, s);
}

int step_tile_width() { return TX; }

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

}  // namespace ssx
