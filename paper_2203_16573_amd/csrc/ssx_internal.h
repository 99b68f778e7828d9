// Internal declarations shared by the host API (ssx_api.cpp) and the HIP
// kernels (ssx_step.hip, ssx_slab.hip, ssx_vec.hip, ssx_grad.hip).  Not part
// of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace ssx {

// Ghost cells around every stored field: always zero, never written, so the
// stencils read "zero outside the grid" without bounds checks.  GX columns
// (also keeps row starts 256-byte aligned for FP32) and GZ rows.  The row
// pitch is at least NX + 2 GX + 8, a multiple of 64.
constexpr int GX = 64;
constexpr int GZ = 8;
// The absorbing-layer factor arrays along z are padded by PZ entries of 1 on
// both sides (the arrays along x are pitch long, origin GX, 1 outside the
// grid), so any tile row or staged halo row reads a factor without a test.
constexpr int PZ = 64;

enum class Dt : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3 };

// Geometry of one padded grid as the kernels see it.
struct GridDims {
  int NZ, NX;              // computational grid (physical + 2 L)
  int L;                   // absorbing layer width (cells)
  int pitch;               // row pitch of field arrays (elements)
  long long field_stride;  // elements between consecutive shots of one field
  long long origin;        // offset of element (0,0) from the array start
};

// A line that is sampled or injected: one or two grid rows with linear
// interpolation weights, ntr consecutive columns.
struct LineDev {
  int row0, row1;   // row1 == row0 with w1 == 0 for a single row
  double w0, w1;
  int col0, ntr;
};

// Per-launch trace I/O: pointer to [shot][nt][ntr] traces, time index, and a
// scale applied to the values (traces are V = double or float).
struct TraceIO {
  const void* in;   // injected traces (nullptr: none)
  void* out;        // sampled traces (nullptr: none)
  int n;            // time index (-1: nothing this launch)
  long long shot_stride;  // nt * ntr
  double scale;
  // per-shot power-of-two field scale (nullptr: 1): injections are divided
  // by dyn[shot], samples multiplied by it (keeps 16-bit fields in range)
  const float* dyn;
};

struct Coef {
  // dt kappa / (h Z0), compute type, laid out like one shot of a field
  // (element (I, J) at origin + I * pitch + J, zero ghosts)
  const void* ck;
  // absorbing-layer factors, compute type: ax_n bx_n ax_h bx_h, each pitch
  // long with element J at GX + J; then az_n bz_n az_h bz_h, each NZ + 2 PZ
  // long with element I at PZ + I (1 outside the grid)
  const void* pml;
  double cb;        // Z0 dt / (rho h) (constant density)
  // variable density: Z0 dt / (rho_x h) at every v_x cell (i, j+1/2) and
  // Z0 dt / (rho_z h) at every v_z cell (i+1/2, j), compute type, laid out
  // like ck; null for constant density (cb is used)
  const void* cbx;
  const void* cbz;
};

// Field pointers of one grid (all shots): main pressure, v_x, v_z and the
// absorbing-layer auxiliary (forward: p_x; transpose: P~x - P~z).
struct Fields {
  void* p;
  void* vx;
  void* vz;
  void* aux;
};

// Everything one fused time-step launch needs: fields at step n (in) and
// n+1 (out), the grid, coefficients and the four line I/O slots.
struct StepArgs {
  Fields in, out;
  GridDims g;
  Coef c;
  LineDev vsl, vil, psl, pil;  // velocity-phase sample/inject, pressure-phase sample/inject
  TraceIO vs, vi, ps, pi;
  int ntx, ntz, nshots;        // tiles across x, down z; shots
  int nt;                      // record length (trace indices outside [0, nt) are skipped)
  int dir;                     // +1 forward, -1 transposed: trace index of level t = n + dir t
  // tile-loop launches of the one-step kernel: per-shot tile indices
  // (tz-row * ntx + tx-column), the ngen general tiles first, then the nint
  // interior ones (see step_tile_lists)
  const int* tiles;
  int ngen, nint;
  // forward one-step launches of the fused kernel may also store the
  // residual of the pressure update of every physical cell (the misfit
  // gradient's step history, GradRows layout); null otherwise
  void* hist;
};

// Rows of the misfit gradient's step history and accumulator: the physical
// columns of a row in the grid's aligned groups of four, group gi covering
// columns 4 (g0 + gi) .. 4 (g0 + gi) + 3 with g0 = L / 4 (entries of
// columns outside the physical grid hold zero).
struct GradRows {
  int g0, ng;  // first group, groups per row
  __host__ __device__ GradRows(int L, int nx) : g0(L / 4), ng((L + nx - 1) / 4 - L / 4 + 1) {}
  __host__ __device__ int width() const { return 4 * ng; }
};

// ---- launchers (ssx_step.hip, ssx_slab.hip) ------------------------------
// One fused time step (velocity then pressure, one launch).  tz: tile height
// (8, 16 or 32; 32 is not available for FP64 fields).  loop: 0, one tile
// per workgroup; else one workgroup per general tile and, for the interior
// tiles (a.tiles lists), a set of workgroups taking several tiles in turn:
// as many as the device holds at once (loop = 1), or at most loop rounded
// down to a multiple of 8 (loop >= 8).
hipError_t launch_step(Dt dt, int order, bool adj, int tz, int loop, StepArgs a, hipStream_t s);
// The tiles of one shot of a grid for the one-step kernel with tile height
// tz, split into those that take the general path (absorbing frame, grid
// edges, rows of any of the given lines) and the interior ones, each list in
// row-major tile order.  Lines count as active at every step, so every
// listed interior tile is interior at every step.
void step_tile_lists(int order, int tz, const GridDims& g, const LineDev* const* lines,
                     int nlines, std::vector<int>* gen, std::vector<int>* inter);
int step_tile_width();
// Heterogeneous batch: up to BATCH_MAX grids (any sizes and records, one
// stencil order and field type, all constant density or all density arrays)
// advanced by one time step in one launch of the fused kernel at tile height
// BATCH_TZ, one tile per workgroup.  Grid p takes blocks [pre[p], pre[p+1]):
// its tile count ntx * ntz * nshots rounded up to a multiple of 8; a[p] are
// its step arguments as for launch_step (no tile lists, no history).
constexpr int BATCH_MAX = 6;
constexpr int BATCH_TZ = 16;
struct BatchStep {
  int n;
  int pre[BATCH_MAX + 1];
  StepArgs a[BATCH_MAX];
};
hipError_t launch_step_batch(Dt dt, int order, bool adj, bool vr, const BatchStep& b,
                             hipStream_t s);
// Several time steps per launch (ssx_slab.hip): ns steps (2, 4 or 8) on
// strips of wr columns (64 or 128; F64 fields and density arrays, a.c.cbx
// set, 64 only) and windows of at
// most SLAB_MAXZ rows held whole in LDS.  a.ntx must be the strip count
// ceil(NX / slab_strip_width(order, ns, wr)) and a.ntz the window count
// slab_windows(order, ns, NZ): 1 for a grid of at most SLAB_MAXZ rows, else
// windows owning slab_window_rows(order, ns) rows each.
constexpr int SLAB_MAXZ = 56;
hipError_t launch_slab(Dt dt, int order, bool adj, int ns, int wr, StepArgs a, hipStream_t s);
// owned columns per strip (0 for an unsupported combination)
int slab_strip_width(int order, int ns, int wr);
// owned rows per window of a taller grid (<= 0: no windows for ns steps)
int slab_window_rows(int order, int ns);
// windows of a grid of NZ rows (0: too tall for ns steps per launch)
int slab_windows(int order, int ns, int NZ);
// All return hipSuccess or the launch error.
hipError_t launch_vel(Dt dt, int order, bool adj, const Fields& f, const GridDims& g,
                      const Coef& c, const LineDev& samp_line, const TraceIO& samp,
                      const LineDev& inj_line, const TraceIO& inj, int nshots,
                      hipStream_t s);
hipError_t launch_pres(Dt dt, int order, bool adj, const Fields& f, const GridDims& g,
                       const Coef& c, const LineDev& samp_line, const TraceIO& samp,
                       const LineDev& inj_line, const TraceIO& inj, int nshots,
                       hipStream_t s);
// sample a line of the main pressure field into traces (forward final step)
hipError_t launch_sample_p(Dt dt, const Fields& f, const GridDims& g,
                           const LineDev& line, const TraceIO& io, int nshots,
                           hipStream_t s);
// zero n bytes (multiple of 4) at ptr with a fill kernel (safe in graphs)
hipError_t launch_zero(void* ptr, size_t bytes, hipStream_t s);

// Vector kernels; V = double when vdbl, float otherwise.  n = elements per
// shot; vectors of consecutive shots are n apart.
// partial sums: grid (NBLK_DOT, nshots); then final reduction into out[shot*ostride + k].
constexpr int NBLK_DOT = 256;
hipError_t launch_dot3(bool vdbl, const void* x, const void* y, long long n, int nshots,
                       double* partial /*[nshots][NBLK_DOT][3]*/, double* out,
                       int ostride, hipStream_t s);
// out[shot*ostride + 0] = sum x*y only (one product)
hipError_t launch_dot1(bool vdbl, const void* x, const void* y, long long n, int nshots,
                       double* partial, double* out, int ostride, hipStream_t s);
// The same with the partial sums in the library's static device array (no
// allocation, no context): out[shot] for 1 <= nshots <= DOT_SCRATCH_SHOTS.
constexpr int DOT_SCRATCH_SHOTS = 64;
hipError_t launch_dot1_static(bool vdbl, const void* x, const void* y, long long n, int nshots,
                              double* out, hipStream_t s);

// y[shot][t][k] = s * f(k, shot) * x   with f chosen by op:
//   0: |xk - xs|, 1: |xk - xs|^2, 2: (1 + a^2 |xk-xs|^2)^(-1/2), 3: 1
// xk = x0 + k h; xs per shot (device doubles).  scale_dev (optional) holds a
// per-shot extra factor applied as well.
hipError_t launch_diag(bool vdbl, int op, double a, double s, const void* x, void* y,
                       long long nt, int ns, int nshots, double x0, double h,
                       const double* xs_dev, hipStream_t st);
// q += alpha2 * |xk - xs|^pw * p (pw = 1 or 2) with alpha2 =
// alpha2_dev[shot*astride], or alpha2_host when alpha2_dev is null
hipError_t launch_add_penalty(bool vdbl, void* q, const void* p, int pw, const double* alpha2_dev,
                              int astride, double alpha2_host, long long nt, int ns,
                              int nshots, double x0, double h, const double* xs_dev,
                              hipStream_t st);

// PCG scalar block per shot (doubles), see ssx_api.cpp for the layout.
constexpr int SC_N = 16;
// SC_GRNEW, SC_GG, SC_RR are consecutive: they receive dot3(g, r) = (g.r, g.g, r.r).
enum Sc { SC_GR = 0, SC_PQ = 1, SC_A = 2, SC_BETA = 3, SC_GRNEW = 4, SC_GG = 5, SC_RR = 6,
          SC_EE = 7, SC_ALPHA2 = 8, SC_FLAG = 9, SC_GR0 = 10, SC_PQ0 = 11, SC_DD = 12,
          SC_TMP = 15 };
// SC_FLAG bits: 1 breakdown (zero <g,r> or <p,q>), 2 non-finite, 4 exact zero
// residual (converged), 8 a sign change of <g,r> or <p,q> was seen (not fatal)
// a = gr / pq (with breakdown checks), per shot
hipError_t launch_pcg_step_length(double* sc, int nshots, hipStream_t s);
// h += a p; r -= a q (n per shot); e += a Fp (ne per shot, e may be null)
hipError_t launch_pcg_update(bool vdbl, void* h, void* r, const void* p, const void* q,
                             void* e, const void* Fp, long long n, long long ne,
                             const double* sc, int nshots, hipStream_t s);
// beta = grnew / gr; gr = grnew; record history row k (k = 0: start, sets gr0)
hipError_t launch_pcg_record(double* sc, double* hist, int k, int maxit, int nshots,
                             hipStream_t s);
// p = g + beta p
hipError_t launch_pcg_dir(bool vdbl, void* p, const void* g, long long n,
                          const double* sc, int nshots, hipStream_t s);
// alpha2 = (alpha * sqrt(rr / dd))^2 from SC_RR = <r0,r0>, SC_DD = <d,d>, or
// alpha^2 itself when absolute; clears flags and reference signs
hipError_t launch_pcg_init(double* sc, double alpha, bool absolute, int nshots, hipStream_t s);
hipError_t launch_neg_copy(bool vdbl, void* y, const void* x, long long n, hipStream_t s);

// Misfit gradient in kappa (ssx_grad.hip; F64 and F32 fields).  hist and
// acc hold, per shot, the nz physical rows, each in the grid's aligned
// groups of four columns that cover the physical ones: grad_cells(L, nz,
// nx) entries per shot (entries of non-physical columns are zero).
long long grad_cells(int L, int nz, int nx);
// hist[shot] = E_h h^n - D^- v^{n+1/2} from the fields f after step n
// (pi: the pressure-source injection of step n)
hipError_t launch_grad_store(Dt dt, int order, const Fields& f, const GridDims& g, int nz, int nx,
                             const LineDev& pil, const TraceIO& pi, void* hist, int nshots,
                             hipStream_t s);
// acc[shot] += P~ hist[shot], P~ the transposed pressure in f
hipError_t launch_grad_acc(Dt dt, const Fields& f, const GridDims& g, int nz, int nx,
                           const void* hist, double* acc, int nshots, hipStream_t s);
// two steps: acc[shot] += P~_a ha[shot], then += P~_b hb[shot] (P~_a, P~_b
// the transposed pressures in fa, fb)
hipError_t launch_grad_acc2(Dt dt, const Fields& fa, const Fields& fb, const GridDims& g, int nz,
                            int nx, const void* ha, const void* hb, double* acc, int nshots,
                            hipStream_t s);
// out[shot][iz][ix] = acc * scale / ck   (out of the vector type)
hipError_t launch_grad_final(Dt dt, const double* acc, const void* ck, const GridDims& g, int nz,
                             int nx, double scale, void* out, int nshots, hipStream_t s);
// e = a - b, n elements per shot
hipError_t launch_sub(bool vdbl, const void* a, const void* b, void* e, long long n, int nshots,
                      hipStream_t s);

// dyn[shot] = smallest power of two >= max(sa * max|a[shot]|, sb * max|b[shot]|)
// (1 when both are zero); b may be null.  partial: [2][nshots][NBLK_DOT] floats.
hipError_t launch_field_scale(bool vdbl, const void* a, double sa, const void* b, double sb,
                              long long n, int nshots, float* partial, float* dyn,
                              hipStream_t s);

}  // namespace ssx
