// Several time steps per launch on a window of at most SLAB_MAXZ rows.
//
// A thin slab (2 L + |dz| + 1 + 2K rows, under SLAB_MAXZ) is one window: a
// workgroup holds its whole height for a strip of WR columns in LDS and
// advances it NS steps before writing back.  A taller grid is cut into
// windows of SLAB_MAXZ rows that overlap: window w owns OZ rows and reads
// HZ = NS (2K-1) more above and below.  One step of the staggered scheme
// reads 2K-1 cells to either side along each axis (K-1 and K for the
// velocity, K and K-1 for the pressure), so after NS steps the cells at
// least NS (2K-1) from the region's edges are exact; the H columns (HZ rows)
// on each side are recomputed by both neighbours, the W = WR - 2H columns
// and OZ rows in the middle are owned and written back.  Regions that reach
// past the grid keep the cells outside it at zero, as the stored ghost
// cells are; rows outside the region read zero from padding rows.
//
// Every cell update uses the same expressions, in the same order, as the
// split and fused step kernels (values are rounded to the storage type
// wherever those kernels store them), so results are bitwise equal.  The
// transposed step reads P~_x = P~_z + aux in the x-stencil everywhere (aux is
// zero off the absorbing frame), like the fused kernel.
//
// Trace slots use level-0 indices from the host and step t uses n + dir t;
// indices outside [0, nt) are skipped.  Lines are injected in every window
// whose region holds their rows (halo rows included) and sampled by the
// window that owns their first row.
//
// Only the columns the remaining steps still need are exact after each step
// (a cone narrowing by the step's reach on each side); on 64-column strips
// the stencil phases skip, per wavefront, column groups outside that cone.
#include "ssx_cell.h"

#include <type_traits>

namespace ssx {

// threads per workgroup: 1024 (16 wavefronts, 128 registers per lane);
// FP64 fields 512, whose values take two registers each
template <typename C> constexpr int slab_threads() { return sizeof(C) == 8 ? 512 : 1024; }
// LDS row padding (floats) of the x-stencil arrays and, on 64-column strips,
// of the v_z and ck arrays.  On 64-column strips a wavefront's lanes take
// consecutive rows, so the row pitch sets which banks a 16-byte access of
// consecutive lanes hits: 4-column padding (pitch = 4 mod 64 words) measured
// fastest (c2 slab, four steps per launch: 4.07 us per step against 4.59
// with 8 columns and 10.3 with none).
constexpr int SLAB_PADX = 4;
constexpr int SLAB_PADZ = 4;
// s_waitcnt operand: vector memory count 0, the other counters unconstrained
constexpr int VMCNT0 = 0x0F70;

template <int K, int NS, int WR, int NT>
struct SlabShape {
  static constexpr int R = 2 * K - 1;                 // per-step reach in x
  static constexpr int H = (NS * R + 3) / 4 * 4;      // halo columns each side
  static constexpr int W = WR - 2 * H;                // owned columns
  static constexpr int RP = WR + SLAB_PADX;           // LDS pitch, x-stencil arrays
  static constexpr int ZR = SLAB_MAXZ + 2 * K;        // LDS rows, z-stencil arrays
  static constexpr int G = WR / 4;                    // 4-column groups per row
  // loads, stores: task q = row q / G, group q % G (consecutive lanes on
  // consecutive columns), NQ tasks per thread
  static constexpr int NQ = (SLAB_MAXZ * G + NT - 1) / NT;
  // windows of a grid taller than SLAB_MAXZ: halo rows on each side and
  // owned rows (no windows where OZ <= 0)
  static constexpr int HZ = NS * R;
  static constexpr int OZ = SLAB_MAXZ - 2 * HZ;
  // stencil phases.  CONE (64-column strips): wavefront w takes column
  // group w + NWV k, its lanes the rows, so that a whole wavefront skips a
  // group outside the columns the remaining steps still need (the cone
  // that narrows by the step's reach on each side per step).  Otherwise
  // the load mapping.  CONE pads the v_z rows as well, so that lanes on
  // consecutive rows hit different LDS banks (there is no room for that
  // padding in LDS at 128 columns), and keeps ck in registers: each thread
  // updates the same cells at every step.
  static constexpr bool CONE = WR == 64;
  static constexpr int NWV = NT / 64;
  static constexpr int NQS = CONE ? (G + NWV - 1) / NWV : NQ;
  static constexpr int ZP = CONE ? WR + SLAB_PADZ : WR;   // LDS pitch, v_z
  static constexpr int NCK = CONE ? 1 : SLAB_MAXZ * WR;   // LDS ck (pitch WR)
  // CONE: the values sampled on the two lines at each step are kept in LDS
  // and written after the last step (no global store in flight during the
  // steps, whose waits for trace loads would otherwise also wait for it:
  // vector memory operations complete in issue order)
  static constexpr int NOUT = CONE ? 2 * NS * W : 1;
  static_assert(!CONE || SLAB_MAXZ <= 64, "one lane per row");
  static_assert(W > 0 && W % 4 == 0, "strip too narrow for the step count");
  static_assert(H <= GX, "halo wider than the ghost columns");
};

// four values of a storage vector in the compute type
template <typename T, typename C>
__device__ __forceinline__ void cvt4(C (&o)[4], const V4<T>& v) {
#pragma unroll
  for (int i = 0; i < 4; ++i) o[i] = ldc<C>(&v.e[i]);
}

// Logical block index of hardware block b of n: workgroups are dealt to the
// 8 XCDs round-robin, so this gives each XCD a contiguous band of strips,
// and neighbouring strips, which overlap by their halo columns, share an L2.
__device__ __forceinline__ int slab_block(int b, int n) {
  const int per = n >> 3, rem = n & 7, xcd = b & 7;
  return xcd * per + (xcd < rem ? xcd : rem) + (b >> 3);
}

template <int K, int NS, int WR>
int slab_owned_width() {
  return SlabShape<K, NS, WR, 1024>::W;
}

// VR: a density array, the velocity coefficient of every v_x and v_z cell
// read once per launch into registers (64-column strips only)
template <int K, bool ADJ, typename T, int NS, int WR, bool VR = false>
__global__ __launch_bounds__(slab_threads<typename Tr<T>::C>()) void k_slab(StepArgs a) {
  using C = typename Tr<T>::C;
  using V = typename Tr<T>::V;
  constexpr int SLAB_THREADS = slab_threads<C>();
  using S = SlabShape<K, NS, WR, SLAB_THREADS>;
  static_assert(!std::is_same<C, double>::value || S::CONE, "F64 fields: 64-column strips");
  static_assert(!VR || S::CONE, "variable density: 64-column strips");
  constexpr int H = S::H, W = S::W, RP = S::RP, G = S::G, NQ = S::NQ, NQS = S::NQS;
  constexpr int ZP = S::ZP, R = S::R;
  // region rows are 0 .. SLAB_MAXZ-1 (region row I is grid row zr + I)
  // p: rows -K .. SLAB_MAXZ+K-1, columns -4 .. WR+3
  __shared__ __align__(32) C sp[S::ZR * RP];
  // v_x and the absorbing-layer auxiliary: rows 0 .. SLAB_MAXZ-1, columns
  // -4 .. WR+3
  __shared__ __align__(32) C svx[SLAB_MAXZ * RP];
  __shared__ __align__(32) C sau[SLAB_MAXZ * RP];
  // v_z: rows -K .. SLAB_MAXZ+K-1, columns 0 .. WR-1
  __shared__ __align__(32) C svz[S::ZR * ZP];
  // absorbing-layer factors: a_n b_n a_h b_h over the region's columns, then
  // over its rows
  __shared__ __align__(32) C spx[4 * WR];
  __shared__ __align__(32) C spz[4 * SLAB_MAXZ];
  // injected values of the current step on the two rows of the v_z line and
  // of the pressure line, over the region's columns (element 2 WR: a slot
  // that threads without a column write to and nobody reads)
  __shared__ __align__(32) C ssv[2 * WR + 4];
  __shared__ __align__(32) C ssp[2 * WR + 4];
  // ck (not CONE): rows 0 .. SLAB_MAXZ-1, columns 0 .. WR-1
  __shared__ __align__(32) C sck[S::NCK];
  // CONE: sampled values, [line (p line, v_z line)][step][owned column]
  __shared__ C sout[S::NOUT];
  auto P_ = [](int I, int c) { return (I + K) * RP + c + 4; };
  auto X_ = [](int I, int c) { return I * RP + c + 4; };
  auto Z_ = [](int I, int c) { return (I + K) * ZP + c; };

  const int NZ = a.g.NZ, NX = a.g.NX, Pt = a.g.pitch, L = a.g.L;
  // block: shot, then window, then strip (XCD-banded order)
  const int per_shot = a.ntx * a.ntz;
  const int blk = slab_block((int)blockIdx.x, (int)gridDim.x);
  const int shot = blk / per_shot;
  const int wz = (blk - shot * per_shot) / a.ntx;
  const int strip = blk - shot * per_shot - wz * a.ntx;
  const int x0 = strip * W;      // first owned column
  const int xr = x0 - H;         // grid column of region column 0
  // rows: one window holding the whole grid (ntz = 1), or window wz owning
  // rows [z0, z1) with HZ halo rows above and below
  const bool win = a.ntz > 1;
  const int z0 = win ? wz * S::OZ : 0;
  const int z1 = win ? min(z0 + S::OZ, NZ) : NZ;
  const int zr = win ? z0 - S::HZ : 0;  // grid row of region row 0
  const long long base = a.g.origin + (long long)shot * a.g.field_stride;
  const T* pA = static_cast<const T*>(a.in.p) + base;
  const T* vxA = static_cast<const T*>(a.in.vx) + base;
  const T* vzA = static_cast<const T*>(a.in.vz) + base;
  const T* auA = static_cast<const T*>(a.in.aux) + base;
  const C* ckp = static_cast<const C*>(a.c.ck) + a.g.origin;
  const C* pml = static_cast<const C*>(a.c.pml);
  const C cb = C(a.c.cb);
  const int tid = threadIdx.x;
  // Line injections: the first 2 WR threads own one region column of a
  // line's row0 (tid < WR) or row1, and compute the value the line injects
  // there at a step into buf[tid].  The trace load is issued a phase or more
  // before the value is needed (fetch), the value formed and stored when it
  // is (finish), with the arithmetic of line_src_at, so that the memory
  // latency overlaps a stencil phase instead of stalling the step.
  const bool filler = tid < 2 * WR;
  const int fj = tid / WR, fcol = xr + (tid - (tid / WR) * WR);
  auto fetch = [&](const LineDev& l, const TraceIO& io, int idx, bool& on) -> C {
    on = filler && io.in && idx >= 0 && idx < a.nt && fcol >= l.col0 && fcol < l.col0 + l.ntr;
    if (!on) return C(0);
    const V* in = static_cast<const V*>(io.in) + shot * io.shot_stride + (long long)idx * l.ntr +
                  (fcol - l.col0);
    return C(*in);
  };
  // finish() begins by waiting for every vector memory operation issued so
  // far (vmcnt 0): the trace loads it consumes were issued a phase earlier,
  // and the wait, taken on every path, keeps the compiler from assuming a
  // load still in flight on paths that do not read its register and from
  // waiting on it, and on every later memory operation, at an unrelated LDS
  // read.  Every thread stores, to its column or to the unread slot.
  auto finish = [&](const LineDev& l, const TraceIO& io, C raw, bool on, C dyn, C* buf) {
    __builtin_amdgcn_s_waitcnt(VMCNT0);
    const int I = fj ? l.row1 : l.row0;
    const C w = (I == l.row0 ? C(l.w0) : C(0)) + (I == l.row1 ? C(l.w1) : C(0));
    buf[filler ? tid : 2 * WR] = on ? w * (C(io.scale) * raw / dyn) : C(0);
  };

  // ---- issue every load of the launch's start, then zero LDS ----------------
  // absorbing-layer factors: one x entry and one z entry per thread
  static_assert(4 * WR <= SLAB_THREADS && 4 * SLAB_MAXZ <= SLAB_THREADS, "one factor per thread");
  C fx = C(1), fz = C(1);
  if (tid < 4 * WR) {
    const int f = tid / WR, J = xr + (tid - f * WR);
    if (J >= 0 && J < NX) fx = pml[f * Pt + GX + J];
  }
  if (tid < 4 * SLAB_MAXZ) {
    // rows of the region outside the grid are never updated; those within
    // PZ of it read the padding entries of 1
    const int f = tid / SLAB_MAXZ, Ig = zr + (tid - f * SLAB_MAXZ);
    if (Ig >= -PZ && Ig < NZ + PZ) fz = pml[4 * Pt + f * (NZ + 2 * PZ) + PZ + Ig];
  }
  // the region: task q: row q / G, columns 4 (q % G) .. +3; all loads are
  // in flight together and land in registers, in the storage type, until LDS
  // is cleared
  V4<T> lp[NQ], lvx[NQ], lvz[NQ], lau[NQ];
  V4<C> lck[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = tid + SLAB_THREADS * k;
    const int I = q / G, c = 4 * (q - (q / G) * G), J = xr + c, Ig = zr + I;
    if (I < SLAB_MAXZ && Ig >= 0 && Ig < NZ && J < NX) {
      // columns J .. J+3 lie in [-GX, NX + 3) (ghost columns read zero)
      const long long o = (long long)Ig * Pt + J;
      lp[k] = *reinterpret_cast<const V4<T>*>(pA + o);
      lvx[k] = *reinterpret_cast<const V4<T>*>(vxA + o);
      lvz[k] = *reinterpret_cast<const V4<T>*>(vzA + o);
      lau[k] = *reinterpret_cast<const V4<T>*>(auA + o);
      if constexpr (!S::CONE) lck[k] = *reinterpret_cast<const V4<C>*>(ckp + o);
    }
  }
  // CONE: ck (VR: and the velocity coefficients) of the cells this thread
  // updates at every step (row tid & 63 of the region, column group
  // (tid >> 6) + NWV k)
  C ckr[NQS][4], cbxr[NQS][4], cbzr[NQS][4];
  if constexpr (S::CONE) {
    const C* bxp = VR ? static_cast<const C*>(a.c.cbx) + a.g.origin : nullptr;
    const C* bzp = VR ? static_cast<const C*>(a.c.cbz) + a.g.origin : nullptr;
#pragma unroll
    for (int k = 0; k < NQS; ++k) {
      const int g = (tid >> 6) + S::NWV * k, I = tid & 63, Ig = zr + I, J = xr + 4 * g;
#pragma unroll
      for (int e = 0; e < 4; ++e) ckr[k][e] = cbxr[k][e] = cbzr[k][e] = C(0);
      if (g < G && I < SLAB_MAXZ && Ig >= 0 && Ig < NZ && J < NX) {
        const long long o = (long long)Ig * Pt + J;
        const V4<C> v = *reinterpret_cast<const V4<C>*>(ckp + o);
#pragma unroll
        for (int e = 0; e < 4; ++e) ckr[k][e] = v.e[e];
        if constexpr (VR) {
          const V4<C> bx = *reinterpret_cast<const V4<C>*>(bxp + o);
          const V4<C> bz = *reinterpret_cast<const V4<C>*>(bzp + o);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            cbxr[k][e] = bx.e[e];
            cbzr[k][e] = bz.e[e];
          }
        }
      }
    }
  }
  const C dynv = a.vi.in ? dyn_of<C>(a.vi, shot) : C(1);
  const C dynp = a.pi.in ? dyn_of<C>(a.pi, shot) : C(1);
  const C dynvs = a.vs.out ? dyn_of<C>(a.vs, shot) : C(1);
  const C dynps = a.ps.out ? dyn_of<C>(a.ps, shot) : C(1);
  // a sampled value written to a line's trace (the arithmetic of
  // line_out_at, with the field scale read once)
  auto emit = [&](const LineDev& l, const TraceIO& io, int idx, int J, C val, C dyn) {
    V* out = static_cast<V*>(io.out) + shot * io.shot_stride + (long long)idx * l.ntr + (J - l.col0);
    *out = V(C(io.scale) * val * dyn);
  };
  // trace values of the injections: CONE issues every step's loads here,
  // with the strip's (one memory latency per launch); otherwise step 0's
  // here and step t + 1's at the start of step t
  bool onv, onp, onvA[NS], onpA[NS];
  C rv = fetch(a.vil, a.vi, a.vi.n, onv);
  C rp = fetch(a.pil, a.pi, a.pi.n, onp);
  C rvA[NS], rpA[NS];
  if constexpr (S::CONE) {
#pragma unroll
    for (int t = 1; t < NS; ++t) {
      rvA[t] = fetch(a.vil, a.vi, a.vi.n + a.dir * t, onvA[t]);
      rpA[t] = fetch(a.pil, a.pi, a.pi.n + a.dir * t, onpA[t]);
    }
  }
  // padding rows and columns stay zero
  for (int i = tid; i < S::ZR * RP; i += SLAB_THREADS) sp[i] = C(0);
  for (int i = tid; i < SLAB_MAXZ * RP; i += SLAB_THREADS) svx[i] = C(0);
  for (int i = tid; i < SLAB_MAXZ * RP; i += SLAB_THREADS) sau[i] = C(0);
  for (int i = tid; i < S::ZR * ZP; i += SLAB_THREADS) svz[i] = C(0);
  if (tid < 4 * WR) spx[tid] = fx;
  if (tid < 4 * SLAB_MAXZ) spz[tid] = fz;
  __syncthreads();

  // ---- store the region --------------------------------------------------
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = tid + SLAB_THREADS * k;
    const int I = q / G, c = 4 * (q - (q / G) * G), J = xr + c, Ig = zr + I;
    if (I < SLAB_MAXZ && Ig >= 0 && Ig < NZ && J < NX) {
      C v[4];
      cvt4(v, lp[k]);
      st4(sp + P_(I, c), v);
      cvt4(v, lvx[k]);
      st4(svx + X_(I, c), v);
      cvt4(v, lvz[k]);
      st4(svz + Z_(I, c), v);
      cvt4(v, lau[k]);
      st4(sau + X_(I, c), v);
      if constexpr (!S::CONE) {
        cvt4(v, lck[k]);
        st4(sck + I * WR + c, v);
      }
    }
  }
  finish(a.vil, a.vi, rv, onv, dynv, ssv);  // step 0
  finish(a.pil, a.pi, rp, onp, dynp, ssp);
  __syncthreads();

  // CONE: each thread updates the same cells at every step, so it keeps
  // their old velocities, pressure and auxiliary, and its row's z factors,
  // in registers from one step to the next; LDS carries the values that
  // other threads' stencils read (lanes past the last row and groups past
  // the last one read clamped, unused values)
  C ovxr[NQS][4], ovzr[NQS][4], pcr[NQS][4], aur[NQS][4];
  C zf[4];  // a_n b_n a_h b_h of the thread's row
  if constexpr (S::CONE) {
    const int I = min(tid & 63, SLAB_MAXZ - 1);
#pragma unroll
    for (int f = 0; f < 4; ++f) zf[f] = spz[f * SLAB_MAXZ + I];
#pragma unroll
    for (int k = 0; k < NQS; ++k) {
      const int c = 4 * min((tid >> 6) + S::NWV * k, G - 1);
      ld4(ovxr[k], svx + X_(I, c));
      ld4(ovzr[k], svz + Z_(I, c));
      ld4(pcr[k], sp + P_(I, c));
      ld4(aur[k], sau + X_(I, c));
    }
  }

  // lines this window samples: those whose first row it owns (the second
  // row, one below, is exact here at sampling time)
  const bool own_vs = a.vsl.row0 >= z0 && a.vsl.row0 < z1;
  const bool own_ps = a.psl.row0 >= z0 && a.psl.row0 < z1;

  // (CONE: unrolled, so that the per-step trace registers are indexed by
  // constants)
  constexpr int TUNROLL = S::CONE ? NS : 1;
#pragma unroll TUNROLL
  for (int t = 0; t < NS; ++t) {
    const int ivs = a.vs.n + a.dir * t, ips = a.ps.n + a.dir * t;
    // pressure injections of step t (the readers of step t - 1 are past the
    // last barrier), then the trace loads of step t + 1
    if constexpr (S::CONE) {
      if (t > 0) finish(a.pil, a.pi, rpA[t], onpA[t], dynp, ssp);
    } else {
      if (t > 0) finish(a.pil, a.pi, rp, onp, dynp, ssp);
      if (t + 1 < NS) {
        rv = fetch(a.vil, a.vi, a.vi.n + a.dir * (t + 1), onv);
        rp = fetch(a.pil, a.pi, a.pi.n + a.dir * (t + 1), onp);
      }
    }

    // pressure-line sampling (p^n), owned columns
    if (a.vs.out && own_vs && ivs >= 0 && ivs < a.nt && tid < W) {
      const int c = H + tid, J = xr + c;
      if (J < NX && J >= a.vsl.col0 && J < a.vsl.col0 + a.vsl.ntr) {
        const C val = C(a.vsl.w0) * sp[P_(a.vsl.row0 - zr, c)] +
                      C(a.vsl.w1) * sp[P_(a.vsl.row1 - zr, c)];
        if constexpr (S::CONE)
          sout[t * W + tid] = val;
        else
          emit(a.vsl, a.vs, ivs, J, val, dynvs);
      }
    }

    // columns the remaining steps need: p of this step on [plo, phi), the
    // velocities on [plo - K, phi + K - 1) (region columns)
    const int plo = H - (NS - 1 - t) * R, phi = H + W + (NS - 1 - t) * R;

    // ---- velocities ----------------------------------------------------------
#pragma unroll
    for (int k = 0; k < NQS; ++k) {
      int I, c;
      if constexpr (S::CONE) {
        const int g = __builtin_amdgcn_readfirstlane((tid >> 6) + S::NWV * k);
        if (g >= G || 4 * g + 4 <= plo - K || 4 * g >= phi + K - 1) continue;
        I = tid & 63;
        c = 4 * g;
      } else {
        const int q = tid + SLAB_THREADS * k;
        I = q / G;
        c = 4 * (q - (q / G) * G);
      }
      const int J = xr + c, Ig = zr + I;
      if (I >= SLAB_MAXZ || Ig < 0 || Ig >= NZ) continue;
      C w[12];  // p (transposed: P~_z + aux) at region columns c-4 .. c+7
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        C pv[4];
        ld4(pv, sp + P_(I, c - 4 + 4 * j));
        if constexpr (ADJ) {
          C av[4];
          ld4(av, sau + X_(I, c - 4 + 4 * j));
#pragma unroll
          for (int e = 0; e < 4; ++e) pv[e] = pv[e] + av[e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) w[4 * j + e] = pv[e];
      }
      C ovx[4], ovz[4], nvx[4], nvz[4];
      if constexpr (S::CONE) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ovx[e] = ovxr[k][e];
          ovz[e] = ovzr[k][e];
        }
      } else {
        ld4(ovx, svx + X_(I, c));
        ld4(ovz, svz + Z_(I, c));
      }
      C sz[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
      for (int m = 1; m <= K; ++m) {
        C hi[4], lo[4];
        ld4(hi, sp + P_(I + m, c));
        ld4(lo, sp + P_(I + 1 - m, c));
#pragma unroll
        for (int e = 0; e < 4; ++e) sz[e] = acc(sz[e], wst<K, C>(m - 1), hi[e], lo[e]);
      }
      C axh[4], bxh[4];
      ld4(axh, spx + 2 * WR + c);
      ld4(bxh, spx + 3 * WR + c);
      const C azh = S::CONE ? zf[2] : spz[2 * SLAB_MAXZ + I];
      const C bzh = S::CONE ? zf[3] : spz[3 * SLAB_MAXZ + I];
      const C* src_row = Ig == a.vil.row0 ? ssv : (Ig == a.vil.row1 ? ssv + WR : nullptr);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int Je = J + e;
        nvx[e] = ovx[e];
        nvz[e] = ovz[e];
        if (Je >= 0 && Je < NX) {
          C sx = C(0);
#pragma unroll
          for (int m = 1; m <= K; ++m) sx = acc(sx, wst<K, C>(m - 1), w[e + 4 + m], w[e + 5 - m]);
          C cbx = cb, cbz = cb;
          if constexpr (VR) {
            cbx = cbxr[k][e];
            cbz = cbzr[k][e];
          }
          nvx[e] = rnd<T>(upd_v<ADJ>(axh[e], bxh[e], cbx, ovx[e], sx, C(0)));
          const C src = src_row ? src_row[c + e] : C(0);
          nvz[e] = rnd<T>(upd_v<ADJ>(azh, bzh, cbz, ovz[e], sz[e], src));
        }
      }
      st4(svx + X_(I, c), nvx);
      st4(svz + Z_(I, c), nvz);
      if constexpr (S::CONE) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          ovxr[k][e] = nvx[e];
          ovzr[k][e] = nvz[e];
        }
      }
      // one task at a time: interleaving two tasks' loads spills registers
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();

    // velocity injections of step t + 1 (read after the next barrier); before
    // the sampling store below, so that waiting for the trace loads does not
    // also wait for that store
    if constexpr (S::CONE) {
      if (t + 1 < NS) finish(a.vil, a.vi, rvA[t + 1], onvA[t + 1], dynv, ssv);
    } else {
      if (t + 1 < NS) finish(a.vil, a.vi, rv, onv, dynv, ssv);
    }

    // v_z-line sampling (v^{n+1/2}), owned columns
    if (a.ps.out && own_ps && ips >= 0 && ips < a.nt && tid < W) {
      const int c = H + tid, J = xr + c;
      if (J < NX && J >= a.psl.col0 && J < a.psl.col0 + a.psl.ntr) {
        const C val = C(a.psl.w0) * svz[Z_(a.psl.row0 - zr, c)] +
                      C(a.psl.w1) * svz[Z_(a.psl.row1 - zr, c)];
        if constexpr (S::CONE)
          sout[(NS + t) * W + tid] = val;
        else
          emit(a.psl, a.ps, ips, J, val, dynps);
      }
    }

    // ---- pressure --------------------------------------------------------------
#pragma unroll
    for (int k = 0; k < NQS; ++k) {
      int I, c;
      if constexpr (S::CONE) {
        const int g = __builtin_amdgcn_readfirstlane((tid >> 6) + S::NWV * k);
        if (g >= G || 4 * g + 4 <= plo || 4 * g >= phi) continue;
        I = tid & 63;
        c = 4 * g;
      } else {
        const int q = tid + SLAB_THREADS * k;
        I = q / G;
        c = 4 * (q - (q / G) * G);
      }
      const int J = xr + c, Ig = zr + I;
      if (I >= SLAB_MAXZ || Ig < 0 || Ig >= NZ) continue;
      C w[12];  // v_x at region columns c-4 .. c+7
      ld4(*reinterpret_cast<C(*)[4]>(w), svx + X_(I, c - 4));
      ld4(*reinterpret_cast<C(*)[4]>(w + 4), svx + X_(I, c));
      ld4(*reinterpret_cast<C(*)[4]>(w + 8), svx + X_(I, c + 4));
      C dx[4] = {C(0), C(0), C(0), C(0)}, dz[4] = {C(0), C(0), C(0), C(0)};
#pragma unroll
      for (int m = 1; m <= K; ++m) {
        C hi[4], lo[4];
        ld4(hi, svz + Z_(I + m - 1, c));
        ld4(lo, svz + Z_(I - m, c));
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          dx[e] = acc(dx[e], wst<K, C>(m - 1), w[e + m + 3], w[e + 4 - m]);
          dz[e] = acc(dz[e], wst<K, C>(m - 1), hi[e], lo[e]);
        }
      }
      C pc[4], pn[4], au[4], an[4], ck[4], axn[4], bxn[4];
      if constexpr (S::CONE) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          pc[e] = pcr[k][e];
          au[e] = aur[k][e];
          ck[e] = ckr[k][e];
        }
      } else {
        ld4(pc, sp + P_(I, c));
        ld4(ck, sck + I * WR + c);
        ld4(au, sau + X_(I, c));
      }
      ld4(axn, spx + c);
      ld4(bxn, spx + WR + c);
      const C azn = S::CONE ? zf[0] : spz[I];
      const C bzn = S::CONE ? zf[1] : spz[SLAB_MAXZ + I];
      const C* src_row = Ig == a.pil.row0 ? ssp : (Ig == a.pil.row1 ? ssp + WR : nullptr);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int Je = J + e;
        pn[e] = pc[e];
        an[e] = au[e];
        if (Je >= 0 && Je < NX) {
          const C src = src_row ? src_row[c + e] : C(0);
          const bool frame = Ig < L || Ig >= NZ - L || Je < L || Je >= NX - L;
          if (!frame) {
            pn[e] = rnd<T>(upd_p<ADJ>(ck[e], pc[e], dx[e], dz[e], src));
          } else {
            C anew;
            pn[e] = rnd<T>(upd_p_frame<ADJ>(ck[e], pc[e], au[e], dx[e], dz[e], src,
                                            axn[e], bxn[e], azn, bzn, &anew));
            an[e] = rnd<T>(anew);
          }
        }
      }
      st4(sp + P_(I, c), pn);
      st4(sau + X_(I, c), an);
      if constexpr (S::CONE) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          pcr[k][e] = pn[e];
          aur[k][e] = an[e];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();
  }

  // ---- CONE: the sampled values (the same tests as at sampling time) ----------
  if constexpr (S::CONE) {
    for (int i = tid; i < 2 * NS * W; i += SLAB_THREADS) {
      const int line = i / (NS * W), t = (i / W) % NS, col = i % W;
      const LineDev& l = line ? a.psl : a.vsl;
      const TraceIO& io = line ? a.ps : a.vs;
      const int idx = io.n + a.dir * t, J = xr + H + col;
      if (io.out && (line ? own_ps : own_vs) && idx >= 0 && idx < a.nt && J < NX &&
          J >= l.col0 && J < l.col0 + l.ntr)
        emit(l, io, idx, J, sout[i], line ? dynps : dynvs);
    }
  }

  // ---- write the owned cells ---------------------------------------------------
  T* pB = static_cast<T*>(a.out.p) + base;
  T* vxB = static_cast<T*>(a.out.vx) + base;
  T* vzB = static_cast<T*>(a.out.vz) + base;
  T* auB = static_cast<T*>(a.out.aux) + base;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    const int q = tid + SLAB_THREADS * k;
    const int I = q / G, c = 4 * (q - (q / G) * G), J = xr + c, Ig = zr + I;
    if (I >= SLAB_MAXZ || Ig < z0 || Ig >= z1 || c < H || c >= H + W || J >= NX) continue;
    const long long o = (long long)Ig * Pt + J;
    C v[4];
    if (J + 3 < NX) {
      ld4(v, sp + P_(I, c));
      st4(pB + o, v);
      ld4(v, svx + X_(I, c));
      st4(vxB + o, v);
      ld4(v, svz + Z_(I, c));
      st4(vzB + o, v);
      ld4(v, sau + X_(I, c));
      st4(auB + o, v);
    } else {
      for (int e = 0; e < 4 && J + e < NX; ++e) {
        stc(pB + o + e, sp[P_(I, c + e)]);
        stc(vxB + o + e, svx[X_(I, c + e)]);
        stc(vzB + o + e, svz[Z_(I, c + e)]);
        stc(auB + o + e, sau[X_(I, c + e)]);
      }
    }
  }
}

// ---------------------------------------------------------------------------

template <int K, bool ADJ, typename T, int NS, int WR, bool VR = false>
static hipError_t slab_go(const StepArgs& a, hipStream_t s) {
  using C = typename Tr<T>::C;
  using S = SlabShape<K, NS, WR, slab_threads<C>()>;
  // strips and windows as the kernel derives them from the block index
  if (a.ntx != (a.g.NX + S::W - 1) / S::W || a.ntz < 1 || a.nshots < 1)
    return hipErrorInvalidValue;
  if (a.ntz == 1 ? a.g.NZ > SLAB_MAXZ : (S::OZ <= 0 || a.ntz != (a.g.NZ + S::OZ - 1) / S::OZ))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_slab<K, ADJ, T, NS, WR, VR>), dim3(a.ntx * a.ntz * a.nshots),
                     dim3(slab_threads<C>()), 0, s, a);
  return hipGetLastError();
}

// the (steps, strip width) pairs with owned columns left (order 8: 8 steps
// need 128 columns); F64 fields and density arrays 64-column strips only
template <int K, bool ADJ, typename T>
static hipError_t slab_t(int ns, int wr, const StepArgs& a, hipStream_t s) {
  if (a.c.cbx) {
    if (wr != 64) return hipErrorInvalidValue;
    if (ns == 2) return slab_go<K, ADJ, T, 2, 64, true>(a, s);
    if (ns == 4) return slab_go<K, ADJ, T, 4, 64, true>(a, s);
    if constexpr (K == 2) {
      if (ns == 8) return slab_go<K, ADJ, T, 8, 64, true>(a, s);
    }
    return hipErrorInvalidValue;
  }
  if (ns == 2 && wr == 64) return slab_go<K, ADJ, T, 2, 64>(a, s);
  if (ns == 4 && wr == 64) return slab_go<K, ADJ, T, 4, 64>(a, s);
  if constexpr (K == 2) {
    if (ns == 8 && wr == 64) return slab_go<K, ADJ, T, 8, 64>(a, s);
  }
  if constexpr (!std::is_same<T, double>::value) {
    if (ns == 2 && wr == 128) return slab_go<K, ADJ, T, 2, 128>(a, s);
    if (ns == 4 && wr == 128) return slab_go<K, ADJ, T, 4, 128>(a, s);
    if (ns == 8 && wr == 128) return slab_go<K, ADJ, T, 8, 128>(a, s);
  }
  return hipErrorInvalidValue;
}

int slab_strip_width(int order, int ns, int wr) {
  const bool o8 = order == 8;
  if (order != 4 && order != 8) return 0;
  if (ns == 2 && wr == 64) return o8 ? slab_owned_width<4, 2, 64>() : slab_owned_width<2, 2, 64>();
  if (ns == 4 && wr == 64) return o8 ? slab_owned_width<4, 4, 64>() : slab_owned_width<2, 4, 64>();
  if (ns == 8 && wr == 64) return o8 ? 0 : slab_owned_width<2, 8, 64>();
  if (ns == 2 && wr == 128)
    return o8 ? slab_owned_width<4, 2, 128>() : slab_owned_width<2, 2, 128>();
  if (ns == 4 && wr == 128)
    return o8 ? slab_owned_width<4, 4, 128>() : slab_owned_width<2, 4, 128>();
  if (ns == 8 && wr == 128)
    return o8 ? slab_owned_width<4, 8, 128>() : slab_owned_width<2, 8, 128>();
  return 0;
}

int slab_window_rows(int order, int ns) { return SLAB_MAXZ - 2 * ns * (order - 1); }

int slab_windows(int order, int ns, int NZ) {
  if (NZ <= SLAB_MAXZ) return 1;
  const int oz = slab_window_rows(order, ns);
  return oz > 0 ? (NZ + oz - 1) / oz : 0;
}

hipError_t launch_slab(Dt dt, int order, bool adj, int ns, int wr, StepArgs a, hipStream_t s) {
  const bool o8 = (order == 8);
  switch (dt) {
    case Dt::F64:
      if (o8) return adj ? slab_t<4, true, double>(ns, wr, a, s) : slab_t<4, false, double>(ns, wr, a, s);
      return adj ? slab_t<2, true, double>(ns, wr, a, s) : slab_t<2, false, double>(ns, wr, a, s);
    case Dt::F32:
      if (o8) return adj ? slab_t<4, true, float>(ns, wr, a, s) : slab_t<4, false, float>(ns, wr, a, s);
      return adj ? slab_t<2, true, float>(ns, wr, a, s) : slab_t<2, false, float>(ns, wr, a, s);
    case Dt::F16:
      if (o8) return adj ? slab_t<4, true, __half>(ns, wr, a, s) : slab_t<4, false, __half>(ns, wr, a, s);
      return adj ? slab_t<2, true, __half>(ns, wr, a, s) : slab_t<2, false, __half>(ns, wr, a, s);
    case Dt::BF16:
      if (o8)
        return adj ? slab_t<4, true, __hip_bfloat16>(ns, wr, a, s)
                   : slab_t<4, false, __hip_bfloat16>(ns, wr, a, s);
      return adj ? slab_t<2, true, __hip_bfloat16>(ns, wr, a, s)
                 : slab_t<2, false, __hip_bfloat16>(ns, wr, a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace ssx
