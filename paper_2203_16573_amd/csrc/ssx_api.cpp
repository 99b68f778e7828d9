// C ABI of libssx: validation, model/coefficient setup, propagation drivers,
// the thin-slab preconditioner and Algorithm 1 (preconditioned CG), the
// weighted normal equations, the other blocks of the modelling operator,
// Lambda~ and the misfit gradient.
//
// Every numerical step runs in the HIP kernels (ssx_step.hip, ssx_slab.hip,
// ssx_vec.hip, ssx_grad.hip); this file only prepares coefficients (once, in
// FP64 on the host), sequences launches on the context's streams and moves
// scalars/history to the host.
#include "ssx.h"
#include "ssx_internal.h"

#include <algorithm>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

using namespace ssx;

namespace {

thread_local std::string g_err;

ssx_status fail(ssx_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define SSX_HIP(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      g_err = std::string(#expr) + ": " + hipGetErrorString(e_);               \
      return SSX_ERR_HIP;                                                      \
    }                                                                          \
  } while (0)

#define SSX_TRY(expr)                 \
  do {                                \
    ssx_status s_ = (expr);           \
    if (s_ != SSX_OK) return s_;      \
  } while (0)

constexpr int HIST_CAP = 4096;  // maximum PCG iterations with history

size_t dtype_size(int dt) {
  switch (dt) {
    case SSX_F64: return 8;
    case SSX_F32: return 4;
    case SSX_F16: return 2;
    case SSX_BF16: return 2;
  }
  return 0;
}

// Sum of |c_m| of the staggered stencil of the given order.
double stencil_abs_sum(int order) {
  if (order == 4) return 9.0 / 8.0 + 1.0 / 24.0;
  return 1225.0 / 1024.0 + 245.0 / 3072.0 + 49.0 / 5120.0 + 5.0 / 7168.0;
}

// A line at physical depth z on one grid.  node = true: p nodes (row i at
// depth (i - L) h); false: v_z half nodes (row i at depth (i - L + 1/2) h).
bool make_line(double z, double x0, int n, double h, int L, int nz_phys, int nx_phys,
               bool node, LineDev* out, std::string* why) {
  const double u = L + z / h - (node ? 0.0 : 0.5);
  int i0 = (int)std::floor(u + 1e-12);
  double w1 = u - i0;
  if (std::fabs(w1) < 1e-12) w1 = 0.0;
  const int lo = L, hi = node ? L + nz_phys - 1 : L + nz_phys - 2;
  const int i1 = (w1 == 0.0) ? i0 : i0 + 1;
  if (i0 < lo || i1 > hi) {
    *why = "line depth outside the physical grid";
    return false;
  }
  const double j0 = x0 / h;
  if (std::fabs(j0 - std::round(j0)) > 1e-9) {
    *why = "line lateral positions must lie on grid columns";
    return false;
  }
  const int c0 = L + (int)std::lround(j0);
  if (n < 1 || c0 < L || c0 + n - 1 > L + nx_phys - 1) {
    *why = "line extends outside the physical grid";
    return false;
  }
  out->row0 = i0;
  out->row1 = i1;
  out->w0 = 1.0 - w1;
  out->w1 = w1;
  out->col0 = c0;
  out->ntr = n;
  return true;
}

// Rows of the full model used by a thin slab around the line at depth z
// with its datum dz cells away: [i_lo, i_hi] (may extend beyond the model;
// clamped when copying kappa); *z_slab is the line's depth in the slab.
void thin_rows(const ssx_problem& p, double z, int dz, int* i_lo, int* i_hi, double* z_slab) {
  const int k = p.order / 2;
  const int i_s = (int)std::floor(z / p.h + 1e-12);
  const double frac = z / p.h - i_s;
  *i_lo = std::min(i_s, i_s + dz) - k;
  *i_hi = std::max(i_s, i_s + dz) + k + (frac > 1e-12 ? 1 : 0);
  *z_slab = z - (*i_lo) * p.h;
}
// the source-side slab (preconditioner, W_m) and the receiver-side one (W_d)
void slab_rows(const ssx_problem& p, int* i_lo, int* i_hi, double* zs_slab) {
  thin_rows(p, p.z_src, p.slab_dz, i_lo, i_hi, zs_slab);
}
void rslab_rows(const ssx_problem& p, int* i_lo, int* i_hi, double* zr_slab) {
  thin_rows(p, p.z_rec, p.rslab_dz, i_lo, i_hi, zr_slab);
}

ssx_status check_problem(const ssx_problem* pp) {
  if (!pp) return fail(SSX_ERR_ARG, "problem is NULL");
  const ssx_problem& p = *pp;
  if (p.order != 4 && p.order != 8) return fail(SSX_ERR_ARG, "order must be 4 or 8");
  if (p.nz < p.order + 1 || p.nx < p.order + 1)
    return fail(SSX_ERR_ARG, "grid smaller than the stencil");
  if (p.npml < 0) return fail(SSX_ERR_ARG, "npml must be >= 0");
  if (!(p.h > 0) || !(p.dt > 0) || !std::isfinite(p.h) || !std::isfinite(p.dt))
    return fail(SSX_ERR_ARG, "h and dt must be positive");
  if (p.nt < 1 || p.ns < 1 || p.nr < 1 || p.nshots < 1)
    return fail(SSX_ERR_ARG, "nt, ns, nr and nshots must be >= 1");
  if (p.slab_dz == 0) return fail(SSX_ERR_ARG, "slab_dz must be nonzero");
  if (p.npml > 0 && !(p.pml_R > 0 && p.pml_R < 1))
    return fail(SSX_ERR_ARG, "pml_R must be in (0, 1)");
  const bool ok_dt = (p.field_dtype == SSX_F64 && p.vec_dtype == SSX_F64) ||
                     ((p.field_dtype == SSX_F32 || p.field_dtype == SSX_F16 ||
                       p.field_dtype == SSX_BF16) &&
                      p.vec_dtype == SSX_F32);
  if (!ok_dt) return fail(SSX_ERR_ARG, "dtypes must be F64/F64 or {F32,F16,BF16}/F32");
  std::string why;
  LineDev l;
  const int L = p.npml;
  if (!make_line(p.z_src, p.x_src0, p.ns, p.h, L, p.nz, p.nx, true, &l, &why))
    return fail(SSX_ERR_ARG, "source line: " + why);
  if (!make_line(p.z_rec, p.x_rec0, p.nr, p.h, L, p.nz, p.nx, true, &l, &why))
    return fail(SSX_ERR_ARG, "receiver line: " + why);
  int i_lo, i_hi;
  double zs;
  slab_rows(p, &i_lo, &i_hi, &zs);
  const int nzs = i_hi - i_lo + 1;
  if (!make_line(zs, p.x_src0, p.ns, p.h, L, nzs, p.nx, false, &l, &why) ||
      !make_line(zs, p.x_src0, p.ns, p.h, L, nzs, p.nx, true, &l, &why) ||
      !make_line(zs + p.slab_dz * p.h, p.x_src0, p.ns, p.h, L, nzs, p.nx, true, &l, &why) ||
      !make_line(zs + p.slab_dz * p.h, p.x_src0, p.ns, p.h, L, nzs, p.nx, false, &l, &why))
    return fail(SSX_ERR_ARG, "thin slab: " + why);
  if (p.rslab_dz != 0) {
    double zr;
    rslab_rows(p, &i_lo, &i_hi, &zr);
    const int nzr = i_hi - i_lo + 1;
    if (!make_line(zr, p.x_rec0, p.nr, p.h, L, nzr, p.nx, false, &l, &why) ||
        !make_line(zr + p.rslab_dz * p.h, p.x_rec0, p.nr, p.h, L, nzr, p.nx, true, &l, &why) ||
        !make_line(zr + p.rslab_dz * p.h, p.x_rec0, p.nr, p.h, L, nzr, p.nx, false, &l, &why))
      return fail(SSX_ERR_ARG, "receiver-side slab: " + why);
  }
  return SSX_OK;
}

ssx_status check_model(const ssx_problem& p, const double* kappa, double rho, double* cmax) {
  if (!(rho > 0) || !std::isfinite(rho)) return fail(SSX_ERR_ARG, "rho must be positive");
  double kmax = 0;
  const size_t n = (size_t)p.nz * p.nx;
  for (size_t i = 0; i < n; ++i) {
    const double k = kappa[i];
    if (!std::isfinite(k) || !(k > 0)) return fail(SSX_ERR_ARG, "kappa must be finite and > 0");
    kmax = std::max(kmax, k);
  }
  *cmax = std::sqrt(kmax / rho);
  const double bound = 1.0 / (std::sqrt(2.0) * stencil_abs_sum(p.order));
  const double courant = *cmax * p.dt / p.h;
  if (courant > bound) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "Courant number %.4f above the stability bound %.4f",
                  courant, bound);
    return fail(SSX_ERR_CFL, buf);
  }
  return SSX_OK;
}

// Variable density: checks rho like kappa and returns the largest velocity
// sqrt(kappa / rho) and impedance sqrt(kappa rho) of the model.
ssx_status check_model_density(const ssx_problem& p, const double* kappa, const double* rho,
                               double* cmax, double* zmax) {
  double c2 = 0, z2 = 0;
  const size_t n = (size_t)p.nz * p.nx;
  for (size_t i = 0; i < n; ++i) {
    const double k = kappa[i], r = rho[i];
    if (!std::isfinite(k) || !(k > 0)) return fail(SSX_ERR_ARG, "kappa must be finite and > 0");
    if (!std::isfinite(r) || !(r > 0)) return fail(SSX_ERR_ARG, "rho must be finite and > 0");
    c2 = std::max(c2, k / r);
    z2 = std::max(z2, k * r);
  }
  *cmax = std::sqrt(c2);
  *zmax = std::sqrt(z2);
  const double bound = 1.0 / (std::sqrt(2.0) * stencil_abs_sum(p.order));
  const double courant = *cmax * p.dt / p.h;
  if (courant > bound) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "Courant number %.4f above the stability bound %.4f",
                  courant, bound);
    return fail(SSX_ERR_CFL, buf);
  }
  return SSX_OK;
}

// Host-side description of one padded grid and its FP64 coefficients.
struct GridHost {
  int nz, nx, L, NZ, NX, pitch;
  long long field_elems;  // one field of one shot, ghosts included
  long long origin;
  std::vector<double> ck;   // laid out like a field (zero ghosts)
  std::vector<double> pml;  // x arrays of length pitch (origin GX), then z arrays
  // variable density: Z0 dt / (rho h) at the v_x and v_z cells, rho there
  // the mean of its two nodes; laid out like ck (empty: constant density)
  std::vector<double> cbx, cbz;
};

int grid_pitch(int NX) { return ((NX + 2 * GX + 8) + 63) / 64 * 64; }

void build_grid(const ssx_problem& p, const std::vector<double>& kphys, int nz, double Z0,
                double rho, GridHost* g, const std::vector<double>* rphys = nullptr) {
  const int L = p.npml, nx = p.nx;
  g->nz = nz;
  g->nx = nx;
  g->L = L;
  g->NZ = nz + 2 * L;
  g->NX = nx + 2 * L;
  g->pitch = grid_pitch(g->NX);
  g->field_elems = (long long)(g->NZ + 2 * GZ) * g->pitch;
  g->origin = (long long)GZ * g->pitch + GX;
  // model padded by copying the nearest physical value
  double kmax = 0;
  g->ck.assign((size_t)g->field_elems, 0.0);
  for (int I = 0; I < g->NZ; ++I) {
    const int i = std::min(std::max(I - L, 0), nz - 1);
    for (int J = 0; J < g->NX; ++J) {
      const int j = std::min(std::max(J - L, 0), nx - 1);
      const double k = kphys[(size_t)i * nx + j];
      kmax = std::max(kmax, k);
      g->ck[(size_t)(g->origin + (long long)I * g->pitch + J)] = p.dt * k / (p.h * Z0);
    }
  }
  // PML: sigma(d) = smax (d / L)^2, d = cells into the layer;
  // a = (1 - sigma dt / 2) / (1 + sigma dt / 2), b = 1 / (1 + sigma dt / 2)
  double cmax = rphys ? 0.0 : std::sqrt(kmax / rho);
  if (rphys) {
    // variable density (padded by copying the nearest physical value): the
    // velocity coefficients at v_x (I, J+1/2) and v_z (I+1/2, J) from the
    // mean density of their two nodes (the last node's own beyond it)
    auto rho_at = [&](int I, int J) {
      const int i = std::min(std::max(I - L, 0), nz - 1);
      const int j = std::min(std::max(J - L, 0), nx - 1);
      return (*rphys)[(size_t)i * nx + j];
    };
    for (size_t q = 0; q < (size_t)nz * nx; ++q)
      cmax = std::max(cmax, std::sqrt(kphys[q] / (*rphys)[q]));
    g->cbx.assign((size_t)g->field_elems, 0.0);
    g->cbz.assign((size_t)g->field_elems, 0.0);
    for (int I = 0; I < g->NZ; ++I) {
      for (int J = 0; J < g->NX; ++J) {
        const double r0 = rho_at(I, J);
        const double rx = 0.5 * (r0 + rho_at(I, std::min(J + 1, g->NX - 1)));
        const double rz = 0.5 * (r0 + rho_at(std::min(I + 1, g->NZ - 1), J));
        const size_t o = (size_t)(g->origin + (long long)I * g->pitch + J);
        g->cbx[o] = Z0 * p.dt / (rx * p.h);
        g->cbz[o] = Z0 * p.dt / (rz * p.h);
      }
    }
  }
  const double smax = L > 0 ? 3.0 * cmax * std::log(1.0 / p.pml_R) / (2.0 * L * p.h) : 0.0;
  auto ab = [&](double pos, int nphys, double* a, double* b) {
    double d = std::max(std::max((double)L - pos, pos - (double)(L + nphys - 1)), 0.0);
    const double sig = L > 0 ? smax * (d / L) * (d / L) : 0.0;
    const double q = 0.5 * sig * p.dt;
    *a = (1.0 - q) / (1.0 + q);
    *b = 1.0 / (1.0 + q);
  };
  const int NX = g->NX, NZ = g->NZ, PX = g->pitch, ZL = NZ + 2 * PZ;
  g->pml.assign(4 * (size_t)PX + 4 * (size_t)ZL, 1.0);
  double* Q = g->pml.data();
  for (int J = 0; J < NX; ++J) {
    ab(J, nx, &Q[GX + J], &Q[PX + GX + J]);
    ab(J + 0.5, nx, &Q[2 * PX + GX + J], &Q[3 * PX + GX + J]);
  }
  double* Z = Q + 4 * (size_t)PX + PZ;
  for (int I = 0; I < NZ; ++I) {
    ab(I, nz, &Z[I], &Z[ZL + I]);
    ab(I + 0.5, nz, &Z[2 * ZL + I], &Z[3 * ZL + I]);
  }
}

struct Alloc {  // bump allocator over one device block
  char* base = nullptr;
  size_t off = 0, cap = 0;
  void* take(size_t bytes) {
    off = (off + 255) / 256 * 256;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

struct Layout {
  size_t fields_full, fields_slab, coef_full, coef_slab, xs, vec_s, vec_r, sc, partial, hist;
  size_t total;
};

}  // namespace

// the text ssx_last_error returns, for the 3D entry points (ssx3_api.cpp)
namespace ssx {
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace ssx

struct GridDev {
  GridHost host;
  GridDims dims;
  Coef coef;
  Fields fields;   // buffer 0 (also the in-place buffer of the split kernels)
  Fields fields1;  // buffer 1 (fused kernel writes step n+1 here, then swaps)
  void* field_block;
  size_t field_bytes;
  // 16-bit fields: per-shot field scale of the grid's current propagation
  // and its partial maxima ([2][nshots][NBLK_DOT]); one set per grid, so
  // propagations on different grids may run concurrently
  float* dyn = nullptr;
  float* amax_part = nullptr;
  // tile lists of the one-step kernel's tile-loop launches, per tile height
  // 8, 16, 32 (index tz / 16): general tiles, then interior ones
  std::vector<int> tiles_host[3];
  int ngen[3] = {0, 0, 0}, nint[3] = {0, 0, 0};
  int* tiles_dev[3] = {nullptr, nullptr, nullptr};
  // variable density: device copies of the velocity coefficient arrays
  // (allocated for every context, used when the model has a density array)
  void* cbx_dev = nullptr;
  void* cbz_dev = nullptr;
};

// A captured propagation: keyed by the operation and every trace pointer it
// reads or writes, so replays are exact re-runs of the captured launches.
struct GraphEntry {
  int op;
  const void* ptr[4];
  int tile_z, fused, spl, group, strip, loop;
  hipGraphExec_t exec;
  unsigned long long last_use;
};

struct ssx_ctx {
  ssx_problem prob;
  Dt fdt;
  bool vdbl;
  size_t fsz, csz, vsz;
  hipStream_t stream;
  double rho, Z0;
  bool vrho = false;  // density given as an array (velocity coefficients per cell)
  GridDev full, slab;
  LineDev h_line, r_line, f_line, dp_line, dv_line;
  // source-side slab: pressure line at z_s (W_m); receiver-side slab (W_d,
  // present when rslab_dz != 0): normal-load line at z_r, datum lines
  LineDev hp_line;
  bool has_rslab = false;
  GridDev rslab;
  LineDev rf_line, rdp_line, rdv_line;
  // full grid: normal-load line at z_s and normal-velocity line at z_r (V);
  // absent when either depth leaves no v_z row pair inside the grid
  bool has_v = false;
  LineDev fv_line, rv_line;
  double* xs_dev;
  // vectors: [nshots][nt][ns] (s) or [nshots][nt][nr] (r)
  void *r, *g, *p, *q, *t1, *sP, *sV, *sF;  // s-vectors
  void *e, *Fp, *t2;                          // r-vectors
  void *rP, *rV, *rW;  // r-vectors of the weighted entry points (null without rslab)
  double* sc;
  double* partial;
  double* hist;
  void* own = nullptr;  // device block allocated by the library (null if workspace)
  bool graphs = true;
  bool fused = true;
  int tile_z_full = 0, tile_z_slab = 0;  // 0: default
  int spl_full = 1, spl_slab = 1;        // time steps per fused launch
  int group_full = 0, group_slab = 0;    // shots per launch (0: from the cache budget)
  int slab_strip = 0;                    // strip width of the multi-step kernel, slab (0: default)
  int strip_full = 0;                    // the same on the full grid
  int loop_full = 0;                     // full-grid one-step kernel: tile loop (0 off)
  hipStream_t cap_stream = nullptr;      // capture stream (graphs are launched on `run`)
  // stream that propagate() issues on: `stream`, or `aux` while the weighted
  // normal operator runs its model-space term beside the data-space chain
  hipStream_t run = nullptr;
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool overlap = true;                   // SSX_OPT_OVERLAP
  // misfit gradient (allocated on first use): r^n of every step and
  // physical cell, [nt][nshots][nz][nx] in the field type; FP64
  // accumulator [nshots][nz][nx]
  void* ghist = nullptr;
  double* gacc = nullptr;
  std::vector<GraphEntry> graphs_cache;
  unsigned long long use_clock = 0;
};

// One context's part of a merged propagation of a heterogeneous batch: what
// propagate() was asked to run.
struct BatchProp {
  ssx_ctx* c;
  GridDev* gd;
  int op;
  bool adj;
  LineDev vsl, vil, psl, pil;
  TraceIO vs, vi, ps, pi;
};

struct BatchGraphEntry {
  std::vector<const void*> key;
  hipGraphExec_t exec;
  unsigned long long last_use;
};

// A heterogeneous batch: contexts solved together, their propagations
// merged.  During ssx_batch_pcg_solve each context's solve runs on a host
// thread of its own; every propagation it reaches waits at a barrier until
// every solve still running has reached its next one, and the last to arrive
// issues all of them as one merged propagation (one launch per time step
// for up to BATCH_MAX grids) on the shared stream, where stream order keeps
// each context's vector work before and after it.
struct ssx_batch {
  std::vector<ssx_ctx*> ctx;
  hipStream_t stream = nullptr;
  Dt fdt = Dt::F32;
  int order = 0;
  hipStream_t cap = nullptr;
  bool graphs = true;
  std::vector<BatchGraphEntry> graph_cache;
  unsigned long long use_clock = 0;
  std::mutex mu;
  std::condition_variable cv;
  int active = 0;                 // solves still running
  unsigned long long gen = 0;     // merged propagations issued
  std::vector<BatchProp> pending;
  ssx_status merged_status = SSX_OK;
  std::string merged_error;
};

namespace {

thread_local ssx_batch* tl_batch = nullptr;

long long nvec_s(const ssx_problem& p) { return (long long)p.nt * p.ns; }
long long nvec_r(const ssx_problem& p) { return (long long)p.nt * p.nr; }

// Lays out every buffer of a context; with a null base only sizes are computed.
void layout(ssx_ctx* c, const GridHost& fg, const GridHost& sg, const GridHost* rg, char* base,
            size_t* total) {
  const ssx_problem& p = c->prob;
  Alloc a;
  a.base = base;
  const int ns = p.nshots;
  const size_t fsz = dtype_size(p.field_dtype);
  const size_t csz = p.field_dtype == SSX_F64 ? 8 : 4;
  const size_t vsz = dtype_size(p.vec_dtype);
  auto grid = [&](GridDev& gd, const GridHost& gh) {
    gd.field_bytes = 8 * (size_t)ns * gh.field_elems * fsz;
    gd.field_block = a.take(gd.field_bytes);
    char* fb = (char*)gd.field_block;
    const size_t one = (size_t)ns * gh.field_elems * fsz;
    gd.fields.p = fb;
    gd.fields.vx = fb ? fb + one : nullptr;
    gd.fields.vz = fb ? fb + 2 * one : nullptr;
    gd.fields.aux = fb ? fb + 3 * one : nullptr;
    gd.fields1.p = fb ? fb + 4 * one : nullptr;
    gd.fields1.vx = fb ? fb + 5 * one : nullptr;
    gd.fields1.vz = fb ? fb + 6 * one : nullptr;
    gd.fields1.aux = fb ? fb + 7 * one : nullptr;
    gd.dyn = (float*)a.take((size_t)ns * 4);
    gd.amax_part = (float*)a.take((size_t)2 * ns * NBLK_DOT * 4);
    gd.coef.ck = a.take((size_t)gh.field_elems * csz);
    gd.coef.pml = a.take((4 * (size_t)gh.pitch + 4 * (size_t)(gh.NZ + 2 * PZ)) * csz);
    gd.cbx_dev = a.take((size_t)gh.field_elems * csz);
    gd.cbz_dev = a.take((size_t)gh.field_elems * csz);
    for (int i = 0; i < 3; ++i) {
      const int tz = 8 << i;
      const size_t n = (size_t)((gh.NX + step_tile_width() - 1) / step_tile_width()) *
                       ((gh.NZ + tz - 1) / tz);
      gd.tiles_dev[i] = (int*)a.take(n * sizeof(int));
    }
  };
  grid(c->full, fg);
  grid(c->slab, sg);
  if (rg) grid(c->rslab, *rg);
  c->xs_dev = (double*)a.take((size_t)ns * 8);
  const size_t bs = (size_t)ns * nvec_s(p) * vsz, br = (size_t)ns * nvec_r(p) * vsz;
  void** svec[] = {&c->r, &c->g, &c->p, &c->q, &c->t1, &c->sP, &c->sV, &c->sF};
  for (void** v : svec) *v = a.take(bs);
  void** rvec[] = {&c->e, &c->Fp, &c->t2};
  for (void** v : rvec) *v = a.take(br);
  void** wvec[] = {&c->rP, &c->rV, &c->rW};
  for (void** v : wvec) *v = rg ? a.take(br) : nullptr;
  c->sc = (double*)a.take((size_t)ns * SC_N * 8);
  c->partial = (double*)a.take((size_t)ns * NBLK_DOT * 3 * 8);
  c->hist = (double*)a.take((size_t)ns * (HIST_CAP + 1) * 4 * 8);
  *total = a.off + 256;
}

ssx_status upload(GridDev& gd, bool dbl, hipStream_t s) {
  const GridHost& g = gd.host;
  // FP64 arrays as they are, else cast once to FP32
  auto put = [&](const void* dst, const std::vector<double>& src) -> ssx_status {
    if (dbl) {
      SSX_HIP(hipMemcpyAsync(const_cast<void*>(dst), src.data(), src.size() * 8,
                             hipMemcpyHostToDevice, s));
    } else {
      std::vector<float> f(src.begin(), src.end());
      SSX_HIP(hipMemcpyAsync(const_cast<void*>(dst), f.data(), f.size() * 4,
                             hipMemcpyHostToDevice, s));
      SSX_HIP(hipStreamSynchronize(s));  // before f goes out of scope
    }
    return SSX_OK;
  };
  SSX_TRY(put(gd.coef.ck, g.ck));
  SSX_TRY(put(gd.coef.pml, g.pml));
  if (!g.cbx.empty()) {
    SSX_TRY(put(gd.cbx_dev, g.cbx));
    SSX_TRY(put(gd.cbz_dev, g.cbz));
    gd.coef.cbx = gd.cbx_dev;
    gd.coef.cbz = gd.cbz_dev;
  } else {
    gd.coef.cbx = gd.coef.cbz = nullptr;
  }
  SSX_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < 3; ++i) {
    if (gd.tiles_host[i].empty()) continue;
    SSX_HIP(hipMemcpyAsync(gd.tiles_dev[i], gd.tiles_host[i].data(),
                           gd.tiles_host[i].size() * sizeof(int), hipMemcpyHostToDevice, s));
  }
  SSX_HIP(hipStreamSynchronize(s));
  return SSX_OK;
}

void fill_dims(GridDev& gd, int nshots) {
  const GridHost& g = gd.host;
  gd.dims.NZ = g.NZ;
  gd.dims.NX = g.NX;
  gd.dims.L = g.L;
  gd.dims.pitch = g.pitch;
  gd.dims.field_stride = g.field_elems;
  gd.dims.origin = g.origin;
  (void)nshots;
}

// Per-shot field arrays are laid out [field][shot][rows][pitch]; the kernels
// take one base pointer per field and step by field_stride between shots.

TraceIO io_none() {
  TraceIO t;
  t.in = nullptr;
  t.out = nullptr;
  t.n = -1;
  t.shot_stride = 0;
  t.scale = 1.0;
  t.dyn = nullptr;
  return t;
}
TraceIO io_in(const void* in, long long stride, double scale) {
  TraceIO t = io_none();
  t.in = in;
  t.shot_stride = stride;
  t.scale = scale;
  return t;
}
TraceIO io_out(void* out, long long stride, double scale) {
  TraceIO t = io_none();
  t.out = out;
  t.shot_stride = stride;
  t.scale = scale;
  return t;
}

int shot_group(const ssx_ctx* c, const GridDev& gd);

// Strip width of the multi-step kernel: the option, else 64 columns for F64
// fields (LDS) and density arrays, 128 otherwise.
int multi_strip(const ssx_ctx* c, bool full, int spl) {
  (void)spl;
  const int opt = full ? c->strip_full : c->slab_strip;
  if (opt) return opt;
  return (c->fdt == Dt::F64 || c->vrho) ? 64 : 128;
}

// Whether spl steps per launch (2, 4 or 8) on strips of wr columns can run on
// a grid of NZ rows: a strip with owned columns left, 64 columns for F64
// fields and density arrays, and windows with owned rows for a grid taller
// than SLAB_MAXZ.  Sets the error message and returns false otherwise.
bool multi_ok(const ssx_ctx* c, int NZ, int spl, int wr) {
  if (c->vrho && wr != 64)
    return fail(SSX_ERR_ARG, "several steps per launch with a density array take 64-column strips"),
           false;
  if (slab_strip_width(c->prob.order, spl, wr) <= 0)
    return fail(SSX_ERR_ARG, "no owned columns for these steps per launch and strip width"), false;
  if (c->fdt == Dt::F64 && wr != 64)
    return fail(SSX_ERR_ARG, "several steps per launch on F64 fields take 64-column strips"), false;
  if (slab_windows(c->prob.order, spl, NZ) <= 0)
    return fail(SSX_ERR_ARG, "the grid is too tall for these steps per launch"), false;
  return true;
}

int default_tile_z(const ssx_ctx* c, const GridDev& gd) {
  // enough tiles to fill 256 CUs several times over, else shorter tiles
  const long long tiles32 = (long long)((gd.host.NX + 63) / 64) * ((gd.host.NZ + 31) / 32) *
                            shot_group(c, gd);
  if (c->fdt == Dt::F64) return tiles32 >= 1024 ? 16 : 8;
  if (tiles32 >= 1024) return 32;
  return tiles32 >= 256 ? 16 : 8;
}

// One propagation over nt steps, issued on stream s.
//   vs: sampled by the velocity phase (a pressure line)
//   vi: injected by the velocity phase (a v_z line)
//   ps: sampled by the pressure phase (a v_z line)
//   pi: injected by the pressure phase (a pressure line)
// Forward: step n samples vs at n-1 (p^n), injects vi[n], samples ps[n]
// (v^{n+1/2}), injects pi[n]; a last launch samples vs at nt-1.
// Transpose: pi[nt-1] enters first; step n (descending) samples vs[n]
// (the transposed pressure after sample n of the adjoint input entered),
// injects vi[n], samples ps[n] and injects pi[n-1].
// A per-step callback of a propagation: called with the step index and the
// fields of the current group (forward: after step n, holding p^{n+1} and
// v^{n+1/2}; transposed: before step n, holding the transposed state of
// level n+1).  `older` is the other field buffer of the fused kernels,
// which still holds what the step before read (forward: the state before
// step n, p^n and v^{n-1/2}, for n >= 1; transposed: level n+2, before
// every step but the first), else null (the split kernels update in
// place).  Steps then run one per launch.
using StepHook = std::function<ssx_status(int n, const Fields& f, const Fields* older)>;
// the same with the first shot and the shot count of the group
using GroupHook =
    std::function<ssx_status(int n, const Fields& f, const Fields* older, int s0, int gs)>;
// Forward propagations with the fused kernels: where step n stores the
// residual of its pressure update (the step history of the misfit
// gradient, GradRows layout, the group's first shot first).  Steps then run
// one per launch.
using StepHist = std::function<void*(int n)>;
using GroupHist = std::function<void*(int n, int s0)>;

// One propagation of ns shots (a group of the context's shots) whose
// fields start at f0 (step n) and f1 (the second buffer).
ssx_status issue_group(ssx_ctx* c, GridDev& gd, bool adj, const Fields& f0, const Fields& f1,
                       int ns, const LineDev& vsl, TraceIO vs, const LineDev& vil, TraceIO vi,
                       const LineDev& psl, TraceIO ps, const LineDev& pil, TraceIO pi,
                       hipStream_t s, const StepHook* hook = nullptr,
                       const StepHist* hist = nullptr) {
  const int nt = c->prob.nt, order = c->prob.order;
  if (hist && (!c->fused || adj)) return fail(SSX_ERR_ARG, "step history needs fused forward steps");
  if (!c->fused) {
    if (!adj) {
      for (int n = 0; n < nt; ++n) {
        vs.n = (vs.out && n >= 1) ? n - 1 : -1;
        vi.n = vi.in ? n : -1;
        SSX_HIP(launch_vel(c->fdt, order, false, f0, gd.dims, gd.coef, vsl, vs, vil, vi,
                           ns, s));
        ps.n = ps.out ? n : -1;
        pi.n = pi.in ? n : -1;
        SSX_HIP(launch_pres(c->fdt, order, false, f0, gd.dims, gd.coef, psl, ps, pil, pi,
                            ns, s));
        if (hook) SSX_TRY((*hook)(n, f0, nullptr));
      }
      if (vs.out) {
        vs.n = nt - 1;
        SSX_HIP(launch_sample_p(c->fdt, f0, gd.dims, vsl, vs, ns, s));
      }
    } else {
      TraceIO none = io_none();
      pi.n = pi.in ? nt - 1 : -1;
      SSX_HIP(launch_pres(c->fdt, order, true, f0, gd.dims, gd.coef, psl, none, pil, pi,
                          ns, s));
      for (int n = nt - 1; n >= 0; --n) {
        if (hook) SSX_TRY((*hook)(n, f0, nullptr));
        vs.n = vs.out ? n : -1;
        vi.n = vi.in ? n : -1;
        SSX_HIP(launch_vel(c->fdt, order, true, f0, gd.dims, gd.coef, vsl, vs, vil, vi,
                           ns, s));
        ps.n = ps.out ? n : -1;
        pi.n = (pi.in && n >= 1) ? n - 1 : -1;
        SSX_HIP(launch_pres(c->fdt, order, true, f0, gd.dims, gd.coef, psl, ps, pil, pi,
                            ns, s));
      }
    }
    return SSX_OK;
  }
  // fused: one launch per step (or per two steps), ping-pong between the two
  // field buffers
  const bool is_full = (&gd == &c->full);
  const int spl = is_full ? c->spl_full : c->spl_slab;
  const int tz_opt = is_full ? c->tile_z_full : c->tile_z_slab;
  const int tz = tz_opt ? tz_opt : default_tile_z(c, gd);
  StepArgs a;
  a.g = gd.dims;
  a.c = gd.coef;
  a.vsl = vsl;
  a.vil = vil;
  a.psl = psl;
  a.pil = pil;
  a.ntx = (gd.host.NX + step_tile_width() - 1) / step_tile_width();
  a.nshots = ns;
  a.nt = nt;
  a.dir = adj ? -1 : 1;
  a.hist = nullptr;
  // one-step launches on the full grid may loop over tiles (lists built at
  // context creation for tile heights 8, 16, 32)
  const int loop = is_full ? c->loop_full : 0;
  const int li = tz == 8 ? 0 : (tz == 16 ? 1 : 2);
  a.tiles = loop ? gd.tiles_dev[li] : nullptr;
  a.ngen = loop ? gd.ngen[li] : 0;
  a.nint = loop ? gd.nint[li] : 0;
  const int ntz1 = (gd.host.NZ + tz - 1) / tz;
  // multi-step kernel: strip width, owned columns, windows
  const int wr = multi_strip(c, is_full, spl);
  const int wown = spl >= 2 ? slab_strip_width(order, spl, wr) : 0;
  const int nwin = spl >= 2 ? slab_windows(order, spl, gd.host.NZ) : 0;
  if (spl >= 2 && (wown <= 0 || nwin <= 0))
    return fail(SSX_ERR_ARG, "steps per launch not available for this grid");
  Fields buf[2] = {f0, f1};
  int cur = 0;
  // one launch covering `steps` (1, or the multi-step kernel's 2, 4 or 8)
  // steps starting at step n with the given level-0 trace indices
  auto launch = [&](int steps, int ivs, int ivi, int ips, int ipi) -> ssx_status {
    a.in = buf[cur];
    a.out = buf[1 - cur];
    a.vs = vs;
    a.vi = vi;
    a.ps = ps;
    a.pi = pi;
    if (steps >= 2) {
      a.vs.n = ivs;
      a.vi.n = ivi;
      a.ps.n = ips;
      a.pi.n = ipi;
      a.ntz = nwin;
      a.ntx = (gd.host.NX + wown - 1) / wown;
      SSX_HIP(launch_slab(c->fdt, order, adj, steps, wr, a, s));
      a.ntx = (gd.host.NX + step_tile_width() - 1) / step_tile_width();
    } else {
      a.vs.n = (vs.out && ivs >= 0 && ivs < nt) ? ivs : -1;
      a.vi.n = (vi.in && ivi >= 0 && ivi < nt) ? ivi : -1;
      a.ps.n = (ps.out && ips >= 0 && ips < nt) ? ips : -1;
      a.pi.n = (pi.in && ipi >= 0 && ipi < nt) ? ipi : -1;
      a.ntz = ntz1;
      SSX_HIP(launch_step(c->fdt, order, adj, tz, loop, a, s));
    }
    cur = 1 - cur;
    return SSX_OK;
  };
  if (!adj) {
    int n = 0;
    if (hook || hist) {
      for (; n < nt; ++n) {
        a.hist = hist ? (*hist)(n) : nullptr;
        SSX_TRY(launch(1, n - 1, n, n, n));
        a.hist = nullptr;
        if (hook) SSX_TRY((*hook)(n, buf[cur], n >= 1 ? &buf[1 - cur] : nullptr));
      }
    }
    for (; n + spl <= nt; n += spl) SSX_TRY(launch(spl, n - 1, n, n, n));
    for (; n < nt; ++n) SSX_TRY(launch(1, n - 1, n, n, n));
    if (vs.out) {
      vs.n = nt - 1;
      SSX_HIP(launch_sample_p(c->fdt, buf[cur], gd.dims, vsl, vs, ns, s));
    }
  } else {
    TraceIO none = io_none();
    TraceIO p0 = pi;
    p0.n = pi.in ? nt - 1 : -1;
    SSX_HIP(launch_pres(c->fdt, order, true, buf[0], gd.dims, gd.coef, psl, none, pil, p0, ns, s));
    int n = nt - 1;
    if (hook) {
      for (; n >= 0; --n) {
        SSX_TRY((*hook)(n, buf[cur], n < nt - 1 ? &buf[1 - cur] : nullptr));
        SSX_TRY(launch(1, n, n, n, n - 1));
      }
    }
    for (; n - spl + 1 >= 0; n -= spl) SSX_TRY(launch(spl, n, n, n, n - 1));
    for (; n >= 0; --n) SSX_TRY(launch(1, n, n, n, n - 1));
  }
  return SSX_OK;
}


// Shots advanced by one launch on grid gd: the option value, else as many
// as keep one step's algorithmic traffic (6 field values and one
// coefficient per cell and shot) within STEP_SET_BYTES, so that a group's
// fields stay in the 256 MB last-level cache from one step to the next.
constexpr double STEP_SET_BYTES = 176.0 * 1024 * 1024;
int shot_group(const ssx_ctx* c, const GridDev& gd) {
  const int ns = c->prob.nshots;
  const int opt = (&gd == &c->full) ? c->group_full : c->group_slab;
  int g;
  if (opt > 0) {
    g = opt;
  } else {
    const double per_shot = (6.0 * c->fsz + c->csz) * gd.host.NZ * gd.host.NX;
    g = std::max(1, (int)(STEP_SET_BYTES / per_shot));
  }
  if (g >= ns) return ns;
  const int ngroups = (ns + g - 1) / g;  // balanced groups
  return (ns + ngroups - 1) / ngroups;
}

Fields shift_fields(const Fields& f, long long elems, size_t fsz) {
  Fields o;
  o.p = (char*)f.p + elems * fsz;
  o.vx = (char*)f.vx + elems * fsz;
  o.vz = (char*)f.vz + elems * fsz;
  o.aux = (char*)f.aux + elems * fsz;
  return o;
}

TraceIO shift_io(TraceIO t, int s0, size_t vsz) {
  if (t.in) t.in = (const char*)t.in + (long long)s0 * t.shot_stride * vsz;
  if (t.out) t.out = (char*)t.out + (long long)s0 * t.shot_stride * vsz;
  if (t.dyn) t.dyn += s0;
  return t;
}

// Start of every propagation: both field buffers zeroed; with 16-bit fields
// the injected traces normalised per shot by a power of two (the trace slots
// then carry the per-shot scales).
ssx_status propagation_start(ssx_ctx* c, GridDev& gd, TraceIO& vs, TraceIO& vi, TraceIO& ps,
                             TraceIO& pi, hipStream_t s) {
  SSX_HIP(launch_zero(gd.field_block, gd.field_bytes, s));
  if (c->fsz == 2) {
    const void* ia = pi.in ? pi.in : vi.in;
    const double sa = pi.in ? pi.scale : vi.scale;
    const void* ib = (pi.in && vi.in) ? vi.in : nullptr;
    const long long nin = (pi.in ? pi.shot_stride : vi.shot_stride);
    if (ia) {
      if (ib && vi.shot_stride != nin) return fail(SSX_ERR_ARG, "mismatched trace inputs");
      SSX_HIP(launch_field_scale(c->vdbl, ia, sa, ib, vi.scale, nin, c->prob.nshots,
                                 gd.amax_part, gd.dyn, s));
      vs.dyn = vi.dyn = ps.dyn = pi.dyn = gd.dyn;
    }
  }
  return SSX_OK;
}

// One propagation of all shots over nt steps, issued on stream s, group by
// group (each group runs its whole record before the next starts).
ssx_status issue_propagation(ssx_ctx* c, GridDev& gd, bool adj, const LineDev& vsl, TraceIO vs,
                             const LineDev& vil, TraceIO vi, const LineDev& psl, TraceIO ps,
                             const LineDev& pil, TraceIO pi, hipStream_t s,
                             const GroupHook* hook = nullptr, const GroupHist* hist = nullptr) {
  const int ns = c->prob.nshots;
  SSX_TRY(propagation_start(c, gd, vs, vi, ps, pi, s));
  const int G = shot_group(c, gd);
  for (int s0 = 0; s0 < ns; s0 += G) {
    const int gs = std::min(G, ns - s0);
    const long long off = (long long)s0 * gd.dims.field_stride;
    StepHook step_hook;
    if (hook)
      step_hook = [&](int n, const Fields& f, const Fields* older) {
        return (*hook)(n, f, older, s0, gs);
      };
    StepHist step_hist;
    if (hist) step_hist = [&](int n) { return (*hist)(n, s0); };
    SSX_TRY(issue_group(c, gd, adj, shift_fields(gd.fields, off, c->fsz),
                        shift_fields(gd.fields1, off, c->fsz), gs, vsl,
                        shift_io(vs, s0, c->vsz), vil, shift_io(vi, s0, c->vsz), psl,
                        shift_io(ps, s0, c->vsz), pil, shift_io(pi, s0, c->vsz), s,
                        hook ? &step_hook : nullptr, hist ? &step_hist : nullptr));
  }
  return SSX_OK;
}

// a weighted PCG solve replays ten distinct propagations; room for them,
// the Euclidean solve, the other operators and a gradient
constexpr size_t GRAPH_CACHE_MAX = 24;

// Replays the cached graph of (op, key pointers, launch options), or captures
// `issue` (given the stream to issue on) into one on first use; runs it on
// the context's stream.
ssx_status cached_graph(ssx_ctx* c, int op, const void* const key[4], int tz, int spl, int group,
                        int strip, int loop, const std::function<ssx_status(hipStream_t)>& issue) {
  for (GraphEntry& e : c->graphs_cache) {
    if (e.op == op && e.ptr[0] == key[0] && e.ptr[1] == key[1] && e.ptr[2] == key[2] &&
        e.ptr[3] == key[3] && e.tile_z == tz && e.fused == (int)c->fused && e.spl == spl &&
        e.group == group && e.strip == strip && e.loop == loop) {
      e.last_use = ++c->use_clock;
      SSX_HIP(hipGraphLaunch(e.exec, c->run));
      return SSX_OK;
    }
  }
  if (!c->cap_stream) SSX_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  SSX_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  ssx_status st = issue(c->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e1 = hipStreamEndCapture(c->cap_stream, &graph);
  if (st != SSX_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  SSX_HIP(e1);
  hipGraphExec_t exec = nullptr;
  hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  SSX_HIP(e2);
  if (c->graphs_cache.size() >= GRAPH_CACHE_MAX) {
    auto lru = std::min_element(c->graphs_cache.begin(), c->graphs_cache.end(),
                                [](const GraphEntry& x, const GraphEntry& y) {
                                  return x.last_use < y.last_use;
                                });
    (void)hipGraphExecDestroy(lru->exec);
    c->graphs_cache.erase(lru);
  }
  GraphEntry ge;
  ge.op = op;
  for (int i = 0; i < 4; ++i) ge.ptr[i] = key[i];
  ge.tile_z = tz;
  ge.fused = (int)c->fused;
  ge.spl = spl;
  ge.group = group;
  ge.strip = strip;
  ge.loop = loop;
  ge.exec = exec;
  ge.last_use = ++c->use_clock;
  c->graphs_cache.push_back(ge);
  SSX_HIP(hipGraphLaunch(exec, c->run));
  return SSX_OK;
}

// Step arguments of step t of a batch member's propagation: those of the
// one-step launch issue_group makes at that step with every shot in one
// launch, at tile height BATCH_TZ and one tile per workgroup.
StepArgs batch_step_args(const BatchProp& q, int t) {
  const ssx_ctx* c = q.c;
  const GridDev& gd = *q.gd;
  const int nt = c->prob.nt;
  StepArgs a{};
  a.g = gd.dims;
  a.c = gd.coef;
  a.vsl = q.vsl;
  a.vil = q.vil;
  a.psl = q.psl;
  a.pil = q.pil;
  a.ntx = (gd.host.NX + step_tile_width() - 1) / step_tile_width();
  a.ntz = (gd.host.NZ + BATCH_TZ - 1) / BATCH_TZ;
  a.nshots = c->prob.nshots;
  a.nt = nt;
  a.dir = q.adj ? -1 : 1;
  a.tiles = nullptr;
  a.ngen = a.nint = 0;
  a.hist = nullptr;
  // the buffers alternate from the first step; forward step n = t samples
  // level n - 1 and injects at n, transposed step n = nt - 1 - t injects the
  // pressure source at n - 1
  a.in = (t & 1) ? gd.fields1 : gd.fields;
  a.out = (t & 1) ? gd.fields : gd.fields1;
  const int n = q.adj ? nt - 1 - t : t;
  const int ivs = q.adj ? n : n - 1, ivi = n, ips = n, ipi = q.adj ? n - 1 : n;
  auto in_range = [nt](int i) { return i >= 0 && i < nt; };
  a.vs = q.vs;
  a.vi = q.vi;
  a.ps = q.ps;
  a.pi = q.pi;
  a.vs.n = (q.vs.out && in_range(ivs)) ? ivs : -1;
  a.vi.n = (q.vi.in && in_range(ivi)) ? ivi : -1;
  a.ps.n = (q.ps.out && in_range(ips)) ? ips : -1;
  a.pi.n = (q.pi.in && in_range(ipi)) ? ipi : -1;
  return a;
}

// The propagations of several batch members as one: each member's start
// (zeroed fields, 16-bit trace scales, the transposed sweep's first pressure
// update), then for every time step one launch per group of up to BATCH_MAX
// members of one direction and density form whose record is still running,
// then each forward member's sampling of its last level.
ssx_status batch_issue(ssx_batch* b, std::vector<BatchProp> P, hipStream_t s) {
  int maxnt = 0;
  for (BatchProp& q : P) {
    ssx_ctx* c = q.c;
    GridDev& gd = *q.gd;
    SSX_TRY(propagation_start(c, gd, q.vs, q.vi, q.ps, q.pi, s));
    if (q.adj) {
      TraceIO p0 = q.pi;
      p0.n = q.pi.in ? c->prob.nt - 1 : -1;
      SSX_HIP(launch_pres(c->fdt, c->prob.order, true, gd.fields, gd.dims, gd.coef, q.psl,
                          io_none(), q.pil, p0, c->prob.nshots, s));
    }
    maxnt = std::max(maxnt, c->prob.nt);
  }
  for (int t = 0; t < maxnt; ++t) {
    for (int form = 0; form < 4; ++form) {
      const bool adj = form & 1, vr = (form & 2) != 0;
      BatchStep bs{};
      auto flush = [&]() -> ssx_status {
        if (bs.n) SSX_HIP(launch_step_batch(b->fdt, b->order, adj, vr, bs, s));
        bs.n = 0;
        return SSX_OK;
      };
      for (const BatchProp& q : P) {
        if (q.adj != adj || q.c->vrho != vr || t >= q.c->prob.nt) continue;
        if (bs.n == BATCH_MAX) SSX_TRY(flush());
        bs.a[bs.n] = batch_step_args(q, t);
        const StepArgs& a = bs.a[bs.n];
        bs.pre[bs.n + 1] = bs.pre[bs.n] + (a.ntx * a.ntz * a.nshots + 7) / 8 * 8;
        ++bs.n;
      }
      SSX_TRY(flush());
    }
  }
  for (const BatchProp& q : P) {
    if (q.adj || !q.vs.out) continue;
    TraceIO vs = q.vs;
    vs.n = q.c->prob.nt - 1;
    const Fields& f = (q.c->prob.nt & 1) ? q.gd->fields1 : q.gd->fields;
    SSX_HIP(launch_sample_p(q.c->fdt, f, q.gd->dims, q.vsl, vs, q.c->prob.nshots, s));
  }
  return SSX_OK;
}

// Issues the pending propagations as one merged propagation: a cached graph
// keyed by every member's context, operation and trace pointers, captured on
// first use, or plain launches.  Called with the batch lock held.
ssx_status batch_flush(ssx_batch* b) {
  std::vector<BatchProp> P;
  P.swap(b->pending);
  // members in batch order, whatever order their threads arrived in, so
  // that a stage replays one graph
  auto rank = [b](const ssx_ctx* c) {
    return std::find(b->ctx.begin(), b->ctx.end(), c) - b->ctx.begin();
  };
  std::sort(P.begin(), P.end(),
            [&](const BatchProp& x, const BatchProp& y) { return rank(x.c) < rank(y.c); });
  if (!b->graphs) return batch_issue(b, P, b->stream);
  std::vector<const void*> key;
  for (const BatchProp& q : P) {
    key.push_back(q.c);
    key.push_back(reinterpret_cast<const void*>((intptr_t)q.op));
    key.push_back(q.vs.out);
    key.push_back(q.vi.in);
    key.push_back(q.ps.out);
    key.push_back(q.pi.in);
  }
  for (BatchGraphEntry& e : b->graph_cache) {
    if (e.key == key) {
      e.last_use = ++b->use_clock;
      SSX_HIP(hipGraphLaunch(e.exec, b->stream));
      return SSX_OK;
    }
  }
  if (!b->cap) SSX_HIP(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
  SSX_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
  const ssx_status st = batch_issue(b, P, b->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e1 = hipStreamEndCapture(b->cap, &graph);
  if (st != SSX_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  SSX_HIP(e1);
  hipGraphExec_t exec = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  SSX_HIP(e2);
  if (b->graph_cache.size() >= GRAPH_CACHE_MAX) {
    auto lru = std::min_element(b->graph_cache.begin(), b->graph_cache.end(),
                                [](const BatchGraphEntry& x, const BatchGraphEntry& y) {
                                  return x.last_use < y.last_use;
                                });
    (void)hipGraphExecDestroy(lru->exec);
    b->graph_cache.erase(lru);
  }
  b->graph_cache.push_back({key, exec, ++b->use_clock});
  SSX_HIP(hipGraphLaunch(exec, b->stream));
  return SSX_OK;
}

// Called with the lock held when a member arrives or leaves: once every
// running solve waits at a propagation, issue them and release the waiters.
void batch_maybe_flush(ssx_batch* b) {
  if (b->pending.empty() || (int)b->pending.size() < b->active) return;
  b->merged_status = batch_flush(b);
  b->merged_error = b->merged_status == SSX_OK ? std::string() : g_err;
  ++b->gen;
  b->cv.notify_all();
}

// propagate() of a batch member: wait for the merged propagation.
ssx_status batch_propagate(ssx_batch* b, const BatchProp& q) {
  std::unique_lock<std::mutex> lk(b->mu);
  const unsigned long long my_gen = b->gen;
  b->pending.push_back(q);
  batch_maybe_flush(b);
  b->cv.wait(lk, [&] { return b->gen != my_gen; });
  if (b->merged_status != SSX_OK) g_err = b->merged_error;
  return b->merged_status;
}

// Runs a propagation: replays a cached graph for (op, pointers) when graphs
// are enabled (capturing it on first use), else issues the launches.  For a
// member of a heterogeneous batch being solved, it joins the batch's next
// merged propagation instead.
ssx_status propagate(ssx_ctx* c, int op, GridDev& gd, bool adj, const LineDev& vsl, TraceIO vs,
                     const LineDev& vil, TraceIO vi, const LineDev& psl, TraceIO ps,
                     const LineDev& pil, TraceIO pi) {
  if (tl_batch)
    return batch_propagate(tl_batch, BatchProp{c, &gd, op, adj, vsl, vil, psl, pil, vs, vi, ps, pi});
  if (!c->graphs)
    return issue_propagation(c, gd, adj, vsl, vs, vil, vi, psl, ps, pil, pi, c->run);
  const void* key[4] = {vs.out, vi.in, ps.out, pi.in};
  const bool full = &gd == &c->full;
  return cached_graph(c, op, key, full ? c->tile_z_full : c->tile_z_slab,
                      full ? c->spl_full : c->spl_slab, full ? c->group_full : c->group_slab,
                      full ? c->strip_full : c->slab_strip, full ? c->loop_full : 0,
                      [&](hipStream_t s) {
                        return issue_propagation(c, gd, adj, vsl, vs, vil, vi, psl, ps, pil, pi,
                                                 s);
                      });
}

void drop_graphs(ssx_ctx* c) {
  for (GraphEntry& e : c->graphs_cache) (void)hipGraphExecDestroy(e.exec);
  c->graphs_cache.clear();
}

enum {
  OP_FWD = 0, OP_ADJ = 1, OP_SLAB_FWD = 2, OP_SLAB_ADJ = 3,
  OP_RSLAB_FWD = 4, OP_RSLAB_ADJ = 5, OP_SLABP_FWD = 6, OP_SLABP_ADJ = 7,
  OP_V_FWD = 8, OP_V_ADJ = 9, OP_LAM_ADJ = 10, OP_LAMT_ADJ = 11, OP_RLAM_ADJ = 12,
  OP_RLAMT_ADJ = 13, OP_TR_INV = 14,
  OP_B01_FWD = 15, OP_B01_ADJ = 16, OP_B10_FWD = 17, OP_B10_ADJ = 18,
  OP_GRAD = 19
};

// The library's second stream and its events, created on first use (at
// the default priority).
ssx_status ensure_aux(ssx_ctx* c) {
  if (c->aux) return SSX_OK;
  SSX_HIP(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  SSX_HIP(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
  SSX_HIP(hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  return SSX_OK;
}

ssx_status do_fwd(ssx_ctx* c, const void* h, void* d) {
  const ssx_problem& p = c->prob;
  return propagate(c, OP_FWD, c->full, false, c->r_line, io_out(d, nvec_r(p), c->Z0), c->r_line,
                   io_none(), c->r_line, io_none(), c->h_line, io_in(h, nvec_s(p), 1.0));
}

ssx_status do_adj(ssx_ctx* c, const void* r, void* g) {
  const ssx_problem& p = c->prob;
  return propagate(c, OP_ADJ, c->full, true, c->h_line, io_out(g, nvec_s(p), 1.0), c->h_line,
                   io_none(), c->h_line, io_none(), c->r_line, io_in(r, nvec_r(p), c->Z0));
}

ssx_status do_slab_fwd(ssx_ctx* c, const void* f, void* P, void* V) {
  const long long st = nvec_s(c->prob);
  return propagate(c, OP_SLAB_FWD, c->slab, false, c->dp_line, io_out(P, st, c->Z0), c->f_line,
                   io_in(f, st, 1.0 / c->Z0), c->dv_line, io_out(V, st, 1.0), c->dp_line,
                   io_none());
}

ssx_status do_slab_adj(ssx_ctx* c, const void* a, const void* b, void* f) {
  const long long st = nvec_s(c->prob);
  return propagate(c, OP_SLAB_ADJ, c->slab, true, c->dp_line, io_none(), c->dv_line, io_in(b, st, 1.0),
                   c->f_line, io_out(f, st, 1.0 / c->Z0), c->dp_line, io_in(a, st, c->Z0));
}

double slab_scale(const ssx_ctx* c) { return c->prob.slab_dz > 0 ? 4.0 : -4.0; }

ssx_status do_precond(ssx_ctx* c, double alpha_hat, const void* r, void* g) {
  const ssx_problem& p = c->prob;
  SSX_HIP(launch_diag(c->vdbl, 2, alpha_hat, 1.0, r, c->t1, p.nt, p.ns, p.nshots, p.x_src0, p.h,
                      c->xs_dev, c->stream));
  SSX_TRY(do_slab_fwd(c, c->t1, c->sP, c->sV));
  SSX_TRY(do_slab_adj(c, c->sV, c->sP, c->sF));  // J (P, V) = (V, P)
  SSX_HIP(launch_diag(c->vdbl, 2, alpha_hat, slab_scale(c), c->sF, g, p.nt, p.ns, p.nshots,
                      p.x_src0, p.h, c->xs_dev, c->stream));
  return SSX_OK;
}

// q = F^T F p + alpha^2 A^T A p, Fp = F p; alpha^2 from the device scalar
// block (alpha2_dev != null) or the host value.
ssx_status do_normal(ssx_ctx* c, const double* alpha2_dev, double alpha2_host, const void* p,
                     void* q, void* Fp) {
  const ssx_problem& pr = c->prob;
  SSX_TRY(do_fwd(c, p, Fp));
  SSX_TRY(do_adj(c, Fp, q));
  SSX_HIP(launch_add_penalty(c->vdbl, q, p, 2, alpha2_dev, SC_N, alpha2_host, pr.nt, pr.ns,
                             pr.nshots, pr.x_src0, pr.h, c->xs_dev, c->stream));
  return SSX_OK;
}

// y = W_d r on the receiver-side slab: X_r r = (P, V) with the normal load
// on z_r, then s_r X_r^T (V, P), s_r = 4 sign(rslab_dz) folded into the
// output scale.
ssx_status do_wd(ssx_ctx* c, const void* r, void* y) {
  const long long st = nvec_r(c->prob);
  const double sr = c->prob.rslab_dz > 0 ? 4.0 : -4.0;
  SSX_TRY(propagate(c, OP_RSLAB_FWD, c->rslab, false, c->rdp_line, io_out(c->rP, st, c->Z0),
                    c->rf_line, io_in(r, st, 1.0 / c->Z0), c->rdv_line, io_out(c->rV, st, 1.0),
                    c->rdp_line, io_none()));
  return propagate(c, OP_RSLAB_ADJ, c->rslab, true, c->rdp_line, io_none(), c->rdv_line,
                   io_in(c->rP, st, 1.0), c->rf_line, io_out(y, st, sr / c->Z0), c->rdp_line,
                   io_in(c->rV, st, c->Z0));
}

// y = W_m x on the source-side slab: a pressure source on z_s, datum
// (P, V) exchanged, the transposed sweep read from the pressure-source slot,
// scaled by sign(slab_dz).  Uses sP and sV.
ssx_status do_wm(ssx_ctx* c, const void* x, void* y) {
  const long long st = nvec_s(c->prob);
  const double sm = c->prob.slab_dz > 0 ? 1.0 : -1.0;
  SSX_TRY(propagate(c, OP_SLABP_FWD, c->slab, false, c->dp_line, io_out(c->sP, st, c->Z0),
                    c->dv_line, io_none(), c->dv_line, io_out(c->sV, st, 1.0), c->hp_line,
                    io_in(x, st, 1.0)));
  return propagate(c, OP_SLABP_ADJ, c->slab, true, c->hp_line, io_out(y, st, sm), c->dv_line,
                   io_in(c->sP, st, 1.0), c->dv_line, io_none(), c->dp_line,
                   io_in(c->sV, st, c->Z0));
}

// y = V f: normal load on z_s, normal velocity sampled on z_r (full grid).
ssx_status do_fwd_v(ssx_ctx* c, const void* f, void* y) {
  const ssx_problem& p = c->prob;
  return propagate(c, OP_V_FWD, c->full, false, c->r_line, io_none(), c->fv_line,
                   io_in(f, nvec_s(p), 1.0 / c->Z0), c->rv_line, io_out(y, nvec_r(p), 1.0),
                   c->h_line, io_none());
}

// g = V^T r (inverse = false) or 4 V^T r: r enters the normal-velocity slot
// on z_r, g is read from the normal-load slot on z_s.  (A captured graph
// holds its scales, so the two forms are distinct operations.)
ssx_status do_adj_v(ssx_ctx* c, const void* r, void* g, bool inverse) {
  const ssx_problem& p = c->prob;
  const double scale = inverse ? 4.0 : 1.0;
  return propagate(c, inverse ? OP_TR_INV : OP_V_ADJ, c->full, true, c->h_line, io_none(), c->rv_line,
                   io_in(r, nvec_r(p), 1.0), c->fv_line, io_out(g, nvec_s(p), scale / c->Z0),
                   c->r_line, io_none());
}

// An off-diagonal block of the vector modelling operator on the full grid:
// src 0 pressure source / 1 normal load on z_s, rec 0 pressure / 1 normal
// velocity on z_r (src != rec), or its transpose.
ssx_status do_block(ssx_ctx* c, int src, int rec, bool transpose, const void* x, void* y) {
  const ssx_problem& p = c->prob;
  const long long ss = nvec_s(p), sr = nvec_r(p);
  const int op = src == 0 ? (transpose ? OP_B01_ADJ : OP_B01_FWD)
                          : (transpose ? OP_B10_ADJ : OP_B10_FWD);
  if (!transpose)
    return propagate(c, op, c->full, false, c->r_line,
                     rec == 0 ? io_out(y, sr, c->Z0) : io_none(), c->fv_line,
                     src == 1 ? io_in(x, ss, 1.0 / c->Z0) : io_none(), c->rv_line,
                     rec == 1 ? io_out(y, sr, 1.0) : io_none(), c->h_line,
                     src == 0 ? io_in(x, ss, 1.0) : io_none());
  return propagate(c, op, c->full, true, c->h_line,
                   src == 0 ? io_out(y, ss, 1.0) : io_none(), c->rv_line,
                   rec == 1 ? io_in(x, sr, 1.0) : io_none(), c->fv_line,
                   src == 1 ? io_out(y, ss, 1.0 / c->Z0) : io_none(), c->r_line,
                   rec == 0 ? io_in(x, sr, c->Z0) : io_none());
}

// y = Lambda~ x (transpose: its transpose) on the source-side slab (side 0)
// or the receiver-side one (side 1): 2 s X^T (0, P) or 2 s X^T (V, 0) with
// (P, V) = X x and s = 4 sign(dz) of that slab.
ssx_status do_lambda(ssx_ctx* c, int side, bool transpose, const void* x, void* y) {
  const ssx_problem& p = c->prob;
  const bool src = side == 0;
  GridDev& g = src ? c->slab : c->rslab;
  const LineDev& fl = src ? c->f_line : c->rf_line;
  const LineDev& dp = src ? c->dp_line : c->rdp_line;
  const LineDev& dv = src ? c->dv_line : c->rdv_line;
  void* P = src ? c->sP : c->rP;
  void* V = src ? c->sV : c->rV;
  const long long st = src ? nvec_s(p) : nvec_r(p);
  const double s2 = ((src ? p.slab_dz : p.rslab_dz) > 0 ? 8.0 : -8.0) / c->Z0;
  SSX_TRY(propagate(c, src ? OP_SLAB_FWD : OP_RSLAB_FWD, g, false, dp, io_out(P, st, c->Z0), fl,
                    io_in(x, st, 1.0 / c->Z0), dv, io_out(V, st, 1.0), dp, io_none()));
  if (!transpose)
    return propagate(c, src ? OP_LAM_ADJ : OP_RLAM_ADJ, g, true, dp, io_none(), dv,
                     io_in(P, st, 1.0), fl, io_out(y, st, s2), dp, io_none());
  return propagate(c, src ? OP_LAMT_ADJ : OP_RLAMT_ADJ, g, true, dp, io_none(), dv, io_none(), fl,
                   io_out(y, st, s2), dp, io_in(V, st, c->Z0));
}

// The model-space term of do_normal_w, sF = W_m A p, issued on stream s.
ssx_status wm_term(ssx_ctx* c, const void* p, hipStream_t s) {
  const ssx_problem& pr = c->prob;
  SSX_HIP(launch_diag(c->vdbl, 0, 0.0, 1.0, p, c->t1, pr.nt, pr.ns, pr.nshots, pr.x_src0, pr.h,
                      c->xs_dev, s));
  c->run = s;
  const ssx_status st = do_wm(c, c->t1, c->sF);
  c->run = c->stream;
  return st;
}

// q = F^T W_d F p + alpha^2 A^T W_m A p, Fp = F p (the W_m term only when
// with_m); alpha^2 as in do_normal.  The W_m term (t1, sF, sP, sV and the
// source-side slab) shares no buffer with the F, W_d, F^T chain (Fp, rW, rP,
// rV, q, the full grid and the receiver-side slab), so with overlap on it
// runs on a second stream, forked after p is ready and joined before the
// two terms are summed; the results do not depend on it.
ssx_status do_normal_w(ssx_ctx* c, const double* alpha2_dev, double alpha2_host, bool with_m,
                       const void* p, void* q, void* Fp) {
  const ssx_problem& pr = c->prob;
  const bool fork = with_m && c->overlap;
  if (fork) {
    // forked after F p, so that W_m's slab simulations run beside W_d's
    // (small grids that leave most of the device idle) rather than beside
    // the full-grid steps
    SSX_TRY(ensure_aux(c));
    SSX_TRY(do_fwd(c, p, Fp));
    SSX_HIP(hipEventRecord(c->ev_fork, c->stream));
    SSX_HIP(hipStreamWaitEvent(c->aux, c->ev_fork, 0));
    ssx_status st = wm_term(c, p, c->aux);
    SSX_HIP(hipEventRecord(c->ev_join, c->aux));
    // the context's stream waits for the second one on every path, so that
    // no work reading p or writing the scratch vectors outlives the call
    if (st == SSX_OK) st = do_wd(c, Fp, c->rW);
    if (st == SSX_OK) st = do_adj(c, c->rW, q);
    SSX_HIP(hipStreamWaitEvent(c->stream, c->ev_join, 0));
    if (st != SSX_OK) return st;
  } else {
    SSX_TRY(do_fwd(c, p, Fp));
    SSX_TRY(do_wd(c, Fp, c->rW));
    SSX_TRY(do_adj(c, c->rW, q));
  }
  if (with_m) {
    if (!fork) SSX_TRY(wm_term(c, p, c->stream));
    SSX_HIP(launch_add_penalty(c->vdbl, q, c->sF, 1, alpha2_dev, SC_N, alpha2_host, pr.nt,
                               pr.ns, pr.nshots, pr.x_src0, pr.h, c->xs_dev, c->stream));
  }
  return SSX_OK;
}

// The device work of one misfit gradient (see ssx_grad.hip) on stream s: a
// forward sweep storing r^n of every step (by the fused step kernel itself,
// else by a kernel after every step), the residual, and a transposed sweep
// accumulating P~^{n+1} r^n before the steps, both one step per launch.
// (Running the side kernels on a second stream beside the next step
// measured slower: the steps already occupy the device.)
ssx_status issue_gradient(ssx_ctx* c, const void* h, const void* d, void* g, hipStream_t s) {
  const ssx_problem& p = c->prob;
  const long long cells = grad_cells(p.npml, p.nz, p.nx);
  const long long ns_ = nvec_s(p), nr_ = nvec_r(p);
  auto hist_at = [&](int n, int s0) {
    return (char*)c->ghist + ((size_t)n * p.nshots + s0) * cells * c->fsz;
  };
  // the fused step kernel stores r^n itself (constant density); the split
  // kernels, and the fused ones with a density array, leave it to a kernel
  // of its own after every step
  const bool hist_fused = c->fused && !c->vrho;
  const GroupHist hist = [&](int n, int s0) -> void* { return hist_at(n, s0); };
  const GroupHook store = [&](int n, const Fields& f, const Fields*, int s0,
                              int gs) -> ssx_status {
    TraceIO pi = shift_io(io_in(h, ns_, 1.0), s0, c->vsz);
    pi.n = n;
    SSX_HIP(launch_grad_store(c->fdt, p.order, f, c->full.dims, p.nz, p.nx, c->h_line, pi,
                              hist_at(n, s0), gs, s));
    return SSX_OK;
  };
  SSX_TRY(issue_propagation(c, c->full, false, c->r_line, io_out(c->Fp, nr_, c->Z0), c->r_line,
                            io_none(), c->r_line, io_none(), c->h_line, io_in(h, ns_, 1.0), s,
                            hist_fused ? nullptr : &store, hist_fused ? &hist : nullptr));
  SSX_HIP(launch_sub(c->vdbl, c->Fp, d, c->e, nr_, p.nshots, s));
  SSX_HIP(launch_dot1(c->vdbl, c->e, c->e, nr_, p.nshots, c->partial, c->sc + SC_TMP, SC_N, s));
  SSX_HIP(launch_zero(c->gacc, (size_t)p.nshots * cells * sizeof(double), s));
  // with the fused kernels' second buffer, steps are accumulated in pairs
  // (n + 1, n) before step n, from the buffer still holding level n + 2 and
  // the current one (the same FP64 sums in the same order, half the
  // accumulator traffic); otherwise one step at a time
  const GroupHook accum = [&](int n, const Fields& f, const Fields* older, int s0,
                              int gs) -> ssx_status {
    double* acc = c->gacc + (size_t)s0 * cells;
    if (!c->fused) {
      SSX_HIP(launch_grad_acc(c->fdt, f, c->full.dims, p.nz, p.nx, hist_at(n, s0), acc, gs, s));
      return SSX_OK;
    }
    const int k = p.nt - 1 - n;  // steps taken so far
    if (k % 2 == 0 && n > 0) return SSX_OK;  // paired with step n - 1
    if (k % 2 == 1) {
      if (!older) return fail(SSX_ERR_ARG, "gradient: no second field buffer");
      SSX_HIP(launch_grad_acc2(c->fdt, *older, f, c->full.dims, p.nz, p.nx, hist_at(n + 1, s0),
                               hist_at(n, s0), acc, gs, s));
    } else {
      SSX_HIP(launch_grad_acc(c->fdt, f, c->full.dims, p.nz, p.nx, hist_at(n, s0), acc, gs, s));
    }
    return SSX_OK;
  };
  SSX_TRY(issue_propagation(c, c->full, true, c->h_line, io_none(), c->h_line, io_none(),
                            c->h_line, io_none(), c->r_line, io_in(c->e, nr_, c->Z0), s, &accum));
  SSX_HIP(launch_grad_final(c->fdt, c->gacc, c->full.coef.ck, c->full.dims, p.nz, p.nx,
                            p.dt / (p.h * c->Z0), g, p.nshots, s));
  return SSX_OK;
}

// g = dJ/dkappa of J = 1/2 ||F h - d||^2 on the physical cells, J per shot,
// replayed as one captured graph when graphs are on.
ssx_status do_gradient(ssx_ctx* c, const void* h, const void* d, void* g, double* J_host) {
  const ssx_problem& p = c->prob;
  const long long cells = grad_cells(p.npml, p.nz, p.nx);
  if (!c->ghist) {
    if (hipMalloc(&c->ghist, (size_t)p.nt * p.nshots * cells * c->fsz) != hipSuccess ||
        hipMalloc((void**)&c->gacc, (size_t)p.nshots * cells * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      if (c->ghist) (void)hipFree(c->ghist);
      c->ghist = nullptr;
      c->gacc = nullptr;
      return fail(SSX_ERR_OOM, "device allocation of the gradient history failed");
    }
  }
  if (!c->graphs) {
    SSX_TRY(issue_gradient(c, h, d, g, c->stream));
  } else {
    const void* key[4] = {h, d, g, nullptr};
    SSX_TRY(cached_graph(c, OP_GRAD, key, c->tile_z_full, c->spl_full, c->group_full, 0,
                         c->loop_full, [&](hipStream_t s) {
                           return issue_gradient(c, h, d, g, s);
                         }));
  }
  if (J_host) {
    std::vector<double> tmp((size_t)p.nshots * SC_N);
    SSX_HIP(hipMemcpyAsync(tmp.data(), c->sc, tmp.size() * 8, hipMemcpyDeviceToHost, c->stream));
    SSX_HIP(hipStreamSynchronize(c->stream));
    for (int sh = 0; sh < p.nshots; ++sh) J_host[sh] = 0.5 * tmp[(size_t)sh * SC_N + SC_TMP];
  }
  return SSX_OK;
}

ssx_status copy_vec(ssx_ctx* c, void* dst, const void* src, size_t bytes) {
  SSX_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
  return SSX_OK;
}

}  // namespace

// ============================================================================
extern "C" {

ssx_status ssx_validate(const ssx_problem* prob, const double* kappa_host, double rho) {
  SSX_TRY(check_problem(prob));
  if (kappa_host) {
    double cmax;
    SSX_TRY(check_model(*prob, kappa_host, rho, &cmax));
  }
  return SSX_OK;
}

size_t ssx_footprint(const ssx_problem* prob) {
  if (check_problem(prob) != SSX_OK) return 0;
  ssx_ctx c{};
  c.prob = *prob;
  int i_lo, i_hi;
  double zs;
  slab_rows(*prob, &i_lo, &i_hi, &zs);
  GridHost fg{}, sg{};
  auto dims = [&](GridHost& g, int nz) {
    g.nz = nz;
    g.nx = prob->nx;
    g.L = prob->npml;
    g.NZ = nz + 2 * g.L;
    g.NX = prob->nx + 2 * g.L;
    g.pitch = grid_pitch(g.NX);
    g.field_elems = (long long)(g.NZ + 2 * GZ) * g.pitch;
  };
  dims(fg, prob->nz);
  dims(sg, i_hi - i_lo + 1);
  GridHost rg{};
  if (prob->rslab_dz != 0) {
    rslab_rows(*prob, &i_lo, &i_hi, &zs);
    dims(rg, i_hi - i_lo + 1);
  }
  size_t total = 0;
  layout(&c, fg, sg, prob->rslab_dz != 0 ? &rg : nullptr, nullptr, &total);
  return total;
}

// ssx_create (rho_host null: constant density rho) and ssx_create_density
// (rho_host: density at every node).
static ssx_status create_impl(const ssx_problem* prob, const double* kappa_host, double rho,
                              const double* rho_host, const double* xs_host, void* stream,
                              void* workspace, size_t workspace_bytes, ssx_ctx** out) {
  if (!out) return fail(SSX_ERR_ARG, "out is NULL");
  *out = nullptr;
  SSX_TRY(check_problem(prob));
  if (!kappa_host || !xs_host) return fail(SSX_ERR_ARG, "kappa_host and xs_host are required");
  double cmax, zmax = 0.0;
  if (rho_host)
    SSX_TRY(check_model_density(*prob, kappa_host, rho_host, &cmax, &zmax));
  else
    SSX_TRY(check_model(*prob, kappa_host, rho, &cmax));
  for (int s = 0; s < prob->nshots; ++s)
    if (!std::isfinite(xs_host[s])) return fail(SSX_ERR_ARG, "xs must be finite");

  ssx_ctx* c = new ssx_ctx();
  c->prob = *prob;
  const ssx_problem& p = c->prob;
  c->fdt = (Dt)p.field_dtype;
  c->vdbl = p.vec_dtype == SSX_F64;
  c->fsz = dtype_size(p.field_dtype);
  c->csz = p.field_dtype == SSX_F64 ? 8 : 4;
  c->vsz = dtype_size(p.vec_dtype);
  c->stream = (hipStream_t)stream;
  c->run = c->stream;
  c->vrho = rho_host != nullptr;
  c->rho = c->vrho ? 0.0 : rho;
  // reference impedance of the stored fields' scaling: rho c_max, or the
  // largest impedance of a density array
  c->Z0 = c->vrho ? zmax : rho * cmax;

  std::vector<double> kphys(kappa_host, kappa_host + (size_t)p.nz * p.nx);
  std::vector<double> rphys;
  if (c->vrho) rphys.assign(rho_host, rho_host + (size_t)p.nz * p.nx);
  // rows i_lo .. i_lo + n - 1 of a model array, clamped to the model
  auto rows_of = [&](const std::vector<double>& m, int i_lo, int n) {
    std::vector<double> out((size_t)n * p.nx);
    for (int r = 0; r < n; ++r) {
      const int i = std::min(std::max(i_lo + r, 0), p.nz - 1);
      std::memcpy(&out[(size_t)r * p.nx], &m[(size_t)i * p.nx], p.nx * sizeof(double));
    }
    return out;
  };
  build_grid(p, kphys, p.nz, c->Z0, rho, &c->full.host, c->vrho ? &rphys : nullptr);
  int i_lo, i_hi;
  double zs;
  slab_rows(p, &i_lo, &i_hi, &zs);
  const int nzs = i_hi - i_lo + 1;
  {
    const std::vector<double> kslab = rows_of(kphys, i_lo, nzs);
    const std::vector<double> rslab = c->vrho ? rows_of(rphys, i_lo, nzs) : std::vector<double>();
    build_grid(p, kslab, nzs, c->Z0, rho, &c->slab.host, c->vrho ? &rslab : nullptr);
  }
  fill_dims(c->full, p.nshots);
  fill_dims(c->slab, p.nshots);
  c->full.coef.cb = c->vrho ? 0.0 : c->Z0 * p.dt / (rho * p.h);
  c->slab.coef.cb = c->full.coef.cb;
  c->has_rslab = p.rslab_dz != 0;
  int r_lo = 0, r_hi = -1;
  double zr = 0.0;
  if (c->has_rslab) {
    rslab_rows(p, &r_lo, &r_hi, &zr);
    const int nzr = r_hi - r_lo + 1;
    const std::vector<double> krs = rows_of(kphys, r_lo, nzr);
    const std::vector<double> rrs = c->vrho ? rows_of(rphys, r_lo, nzr) : std::vector<double>();
    build_grid(p, krs, nzr, c->Z0, rho, &c->rslab.host, c->vrho ? &rrs : nullptr);
    fill_dims(c->rslab, p.nshots);
    c->rslab.coef.cb = c->full.coef.cb;
  }

  std::string why;
  const int L = p.npml;
  make_line(p.z_src, p.x_src0, p.ns, p.h, L, p.nz, p.nx, true, &c->h_line, &why);
  make_line(p.z_rec, p.x_rec0, p.nr, p.h, L, p.nz, p.nx, true, &c->r_line, &why);
  make_line(zs, p.x_src0, p.ns, p.h, L, nzs, p.nx, false, &c->f_line, &why);
  make_line(zs + p.slab_dz * p.h, p.x_src0, p.ns, p.h, L, nzs, p.nx, true, &c->dp_line, &why);
  make_line(zs + p.slab_dz * p.h, p.x_src0, p.ns, p.h, L, nzs, p.nx, false, &c->dv_line, &why);
  make_line(zs, p.x_src0, p.ns, p.h, L, nzs, p.nx, true, &c->hp_line, &why);
  c->has_v = make_line(p.z_src, p.x_src0, p.ns, p.h, L, p.nz, p.nx, false, &c->fv_line, &why) &&
             make_line(p.z_rec, p.x_rec0, p.nr, p.h, L, p.nz, p.nx, false, &c->rv_line, &why);
  if (c->has_rslab) {
    const int nzr = r_hi - r_lo + 1;
    make_line(zr, p.x_rec0, p.nr, p.h, L, nzr, p.nx, false, &c->rf_line, &why);
    make_line(zr + p.rslab_dz * p.h, p.x_rec0, p.nr, p.h, L, nzr, p.nx, true, &c->rdp_line, &why);
    make_line(zr + p.rslab_dz * p.h, p.x_rec0, p.nr, p.h, L, nzr, p.nx, false, &c->rdv_line,
              &why);
  }
  // full-grid tile lists for tile-loop launches (its lines: source and
  // receivers on p nodes and, for V, on v_z nodes)
  {
    const LineDev* lines[4] = {&c->h_line, &c->r_line, &c->fv_line, &c->rv_line};
    const int nlines = c->has_v ? 4 : 2;
    for (int i = 0; i < 3; ++i) {
      std::vector<int> gen, inter;
      step_tile_lists(p.order, 8 << i, c->full.dims, lines, nlines, &gen, &inter);
      c->full.ngen[i] = (int)gen.size();
      c->full.nint[i] = (int)inter.size();
      c->full.tiles_host[i] = gen;
      c->full.tiles_host[i].insert(c->full.tiles_host[i].end(), inter.begin(), inter.end());
    }
  }

  size_t total = 0;
  const GridHost* rg = c->has_rslab ? &c->rslab.host : nullptr;
  layout(c, c->full.host, c->slab.host, rg, nullptr, &total);
  char* base = nullptr;
  if (workspace) {
    if (workspace_bytes < total) {
      delete c;
      return fail(SSX_ERR_OOM, "workspace smaller than ssx_footprint()");
    }
    base = (char*)workspace;
  } else {
    if (hipMalloc((void**)&base, total) != hipSuccess) {
      delete c;
      (void)hipGetLastError();
      return fail(SSX_ERR_OOM, "device allocation of the context failed");
    }
    c->own = base;
  }
  // align the base to 256 bytes
  char* aligned = (char*)(((uintptr_t)base + 255) / 256 * 256);
  layout(c, c->full.host, c->slab.host, rg, aligned, &total);
  ssx_status st = SSX_OK;
  auto cleanup = [&]() {
    if (c->own) (void)hipFree(c->own);
    delete c;
  };
  if (hipMemsetAsync(aligned, 0, total - 256, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->xs_dev, xs_host, p.nshots * sizeof(double), hipMemcpyHostToDevice,
                     c->stream) != hipSuccess) {
    cleanup();
    return fail(SSX_ERR_HIP, "context initialisation failed");
  }
  st = upload(c->full, c->fdt == Dt::F64, c->stream);
  if (st == SSX_OK) st = upload(c->slab, c->fdt == Dt::F64, c->stream);
  if (st == SSX_OK && c->has_rslab) st = upload(c->rslab, c->fdt == Dt::F64, c->stream);
  if (st != SSX_OK) {
    cleanup();
    return st;
  }
  *out = c;
  return SSX_OK;
}

ssx_status ssx_create(const ssx_problem* prob, const double* kappa_host, double rho,
                      const double* xs_host, void* stream, void* workspace,
                      size_t workspace_bytes, ssx_ctx** out) {
  return create_impl(prob, kappa_host, rho, nullptr, xs_host, stream, workspace,
                     workspace_bytes, out);
}

ssx_status ssx_create_density(const ssx_problem* prob, const double* kappa_host,
                              const double* rho_host, const double* xs_host, void* stream,
                              void* workspace, size_t workspace_bytes, ssx_ctx** out) {
  if (!rho_host) return fail(SSX_ERR_ARG, "rho_host is required");
  return create_impl(prob, kappa_host, 0.0, rho_host, xs_host, stream, workspace,
                     workspace_bytes, out);
}

void ssx_destroy(ssx_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->aux) (void)hipStreamSynchronize(c->aux);
  drop_graphs(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux) (void)hipStreamDestroy(c->aux);
  if (c->ghist) (void)hipFree(c->ghist);
  if (c->gacc) (void)hipFree(c->gacc);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->own) (void)hipFree(c->own);
  delete c;
}

ssx_status ssx_fwd(ssx_ctx* c, const void* h, void* d) {
  if (!c || !h || !d) return fail(SSX_ERR_ARG, "null argument");
  return do_fwd(c, h, d);
}

ssx_status ssx_adj(ssx_ctx* c, const void* r, void* g) {
  if (!c || !r || !g) return fail(SSX_ERR_ARG, "null argument");
  return do_adj(c, r, g);
}

ssx_status ssx_slab_fwd(ssx_ctx* c, const void* f, void* P, void* V) {
  if (!c || !f || !P || !V) return fail(SSX_ERR_ARG, "null argument");
  return do_slab_fwd(c, f, P, V);
}

ssx_status ssx_slab_adj(ssx_ctx* c, const void* a, const void* b, void* f) {
  if (!c || !a || !b || !f) return fail(SSX_ERR_ARG, "null argument");
  return do_slab_adj(c, a, b, f);
}

ssx_status ssx_penalty(ssx_ctx* c, int op, double a, const void* x, void* y) {
  if (!c || !x || !y) return fail(SSX_ERR_ARG, "null argument");
  if (op < SSX_PEN_A || op > SSX_PEN_DHALF) return fail(SSX_ERR_ARG, "unknown penalty op");
  if (!std::isfinite(a)) return fail(SSX_ERR_ARG, "a must be finite");
  const ssx_problem& p = c->prob;
  SSX_HIP(launch_diag(c->vdbl, op, a, 1.0, x, y, p.nt, p.ns, p.nshots, p.x_src0, p.h, c->xs_dev,
                      c->stream));
  return SSX_OK;
}

ssx_status ssx_precond(ssx_ctx* c, double alpha_hat, const void* r, void* g) {
  if (!c || !r || !g) return fail(SSX_ERR_ARG, "null argument");
  if (!std::isfinite(alpha_hat)) return fail(SSX_ERR_ARG, "alpha_hat must be finite");
  return do_precond(c, alpha_hat, r, g);
}

ssx_status ssx_normal(ssx_ctx* c, double alpha, const void* p, void* q, void* Fp) {
  if (!c || !p || !q) return fail(SSX_ERR_ARG, "null argument");
  if (!std::isfinite(alpha)) return fail(SSX_ERR_ARG, "alpha must be finite");
  return do_normal(c, nullptr, alpha * alpha, p, q, Fp ? Fp : c->t2);
}

ssx_status ssx_dot(ssx_ctx* c, const void* x, const void* y, int64_t n, double* out_host) {
  if (!c || !x || !y || !out_host || n < 0) return fail(SSX_ERR_ARG, "bad argument");
  const int ns = c->prob.nshots;
  SSX_HIP(launch_dot1(c->vdbl, x, y, n, ns, c->partial, c->sc + SC_TMP, SC_N, c->stream));
  std::vector<double> tmp((size_t)ns * SC_N);
  SSX_HIP(hipMemcpyAsync(tmp.data(), c->sc, tmp.size() * 8, hipMemcpyDeviceToHost, c->stream));
  SSX_HIP(hipStreamSynchronize(c->stream));
  for (int s = 0; s < ns; ++s) out_host[s] = tmp[(size_t)s * SC_N + SC_TMP];
  return SSX_OK;
}

ssx_status ssx_dot_static(const void* x, const void* y, int64_t n, int32_t nshots,
                          int32_t vec_dtype, double* out_dev, void* stream) {
  if (!x || !y || !out_dev || n < 0) return fail(SSX_ERR_ARG, "bad argument");
  if (nshots < 1 || nshots > SSX_DOT_STATIC_MAX_SHOTS)
    return fail(SSX_ERR_ARG, "ssx_dot_static: nshots must lie in [1, " +
                                 std::to_string(SSX_DOT_STATIC_MAX_SHOTS) + "]");
  if (vec_dtype != SSX_F64 && vec_dtype != SSX_F32)
    return fail(SSX_ERR_ARG, "ssx_dot_static: vec_dtype must be SSX_F64 or SSX_F32");
  static_assert(SSX_DOT_STATIC_MAX_SHOTS == DOT_SCRATCH_SHOTS, "scratch size");
  SSX_HIP(launch_dot1_static(vec_dtype == SSX_F64, x, y, n, nshots, out_dev,
                             static_cast<hipStream_t>(stream)));
  return SSX_OK;
}

}  // extern "C"

namespace {

// Algorithm 1 for ssx_pcg_solve (EUCLID: N h = F^T d, alpha =
// a ||F^T d|| / ||d||, alpha_hat = a), ssx_pcg_solve_w (WEIGHTED: N_w h =
// F^T W_d d, alpha = alpha_hat = a) and ssx_pcg_solve_v (VELOCITY: the
// normal load as the unknown, N_v f = V^T d with V in place of F, alpha as
// EUCLID, M = I).
enum class Pcg { EUCLID, WEIGHTED, VELOCITY };
ssx_status run_pcg(ssx_ctx* c, Pcg mode, const void* d, double a, int32_t maxit, double rtol,
                   int32_t use_precond, void* h_out, double* hist_host, int32_t* iters_host) {
  const bool weighted = mode == Pcg::WEIGHTED;
  const ssx_problem& p = c->prob;
  hipStream_t s = c->stream;
  const int ns = p.nshots;
  const long long n = nvec_s(p), ne = nvec_r(p);
  const size_t bs = (size_t)ns * n * c->vsz;
  double* sc = c->sc;
  double* hist = c->hist;
  void* h = h_out;

  SSX_HIP(launch_zero(h, bs, s));
  if (weighted) {  // r_0 = F^T W_d d
    SSX_TRY(do_wd(c, d, c->rW));
    SSX_TRY(do_adj(c, c->rW, c->r));
  } else if (mode == Pcg::VELOCITY) {  // r_0 = V^T d
    SSX_TRY(do_adj_v(c, d, c->r, false));
  } else {  // r_0 = F^T d
    SSX_TRY(do_adj(c, d, c->r));
  }
  SSX_HIP(launch_dot1(c->vdbl, d, d, ne, ns, c->partial, sc + SC_DD, SC_N, s));
  SSX_HIP(launch_dot1(c->vdbl, c->r, c->r, n, ns, c->partial, sc + SC_RR, SC_N, s));
  SSX_HIP(launch_pcg_init(sc, a, weighted, ns, s));
  SSX_HIP(launch_neg_copy(c->vdbl, c->e, d, (long long)ns * ne, s));  // e_0 = F h_0 - d
  auto apply_M = [&](const void* r, void* g) -> ssx_status {
    if (use_precond) return do_precond(c, a, r, g);
    return copy_vec(c, g, r, bs);
  };
  auto apply_N = [&]() -> ssx_status {
    if (weighted) return do_normal_w(c, sc + SC_ALPHA2, 0.0, a != 0.0, c->p, c->q, c->Fp);
    if (mode == Pcg::VELOCITY) {  // q = V^T V p + alpha^2 A^T A p
      SSX_TRY(do_fwd_v(c, c->p, c->Fp));
      SSX_TRY(do_adj_v(c, c->Fp, c->q, false));
      SSX_HIP(launch_add_penalty(c->vdbl, c->q, c->p, 2, sc + SC_ALPHA2, SC_N, 0.0, p.nt, p.ns,
                                 p.nshots, p.x_src0, p.h, c->xs_dev, s));
      return SSX_OK;
    }
    return do_normal(c, sc + SC_ALPHA2, 0.0, c->p, c->q, c->Fp);
  };
  SSX_TRY(apply_M(c->r, c->g));
  SSX_TRY(copy_vec(c, c->p, c->g, bs));
  if (maxit > 0) SSX_TRY(apply_N());
  SSX_HIP(launch_dot3(c->vdbl, c->g, c->r, n, ns, c->partial, sc + SC_GRNEW, SC_N, s));
  SSX_HIP(launch_dot1(c->vdbl, c->e, c->e, ne, ns, c->partial, sc + SC_EE, SC_N, s));
  SSX_HIP(launch_pcg_record(sc, hist, 0, maxit, ns, s));
  int iters = 0;
  std::vector<double> hrow((size_t)ns * SC_N);
  for (int k = 0; k < maxit; ++k) {
    SSX_HIP(launch_dot1(c->vdbl, c->p, c->q, n, ns, c->partial, sc + SC_PQ, SC_N, s));
    SSX_HIP(launch_pcg_step_length(sc, ns, s));
    SSX_HIP(launch_pcg_update(c->vdbl, h, c->r, c->p, c->q, c->e, c->Fp, n, ne, sc, ns, s));
    SSX_TRY(apply_M(c->r, c->g));
    SSX_HIP(launch_dot3(c->vdbl, c->g, c->r, n, ns, c->partial, sc + SC_GRNEW, SC_N, s));
    SSX_HIP(launch_dot1(c->vdbl, c->e, c->e, ne, ns, c->partial, sc + SC_EE, SC_N, s));
    SSX_HIP(launch_pcg_record(sc, hist, k + 1, maxit, ns, s));
    SSX_HIP(launch_pcg_dir(c->vdbl, c->p, c->g, n, sc, ns, s));
    iters = k + 1;
    bool stop = false;
    if (rtol > 0) {
      std::vector<double> rows((size_t)ns * 2);
      for (int sh = 0; sh < ns; ++sh) {
        SSX_HIP(hipMemcpyAsync(&rows[2 * sh], hist + ((size_t)sh * (maxit + 1) + 0) * 4, 8,
                               hipMemcpyDeviceToHost, s));
        SSX_HIP(hipMemcpyAsync(&rows[2 * sh + 1], hist + ((size_t)sh * (maxit + 1) + k + 1) * 4,
                               8, hipMemcpyDeviceToHost, s));
      }
      SSX_HIP(hipStreamSynchronize(s));
      stop = true;
      for (int sh = 0; sh < ns; ++sh)
        if (!(rows[2 * sh + 1] <= rtol * rows[2 * sh])) stop = false;
    }
    if (stop) break;
    if (k < maxit - 1) SSX_TRY(apply_N());
  }
  SSX_HIP(hipMemcpyAsync(hrow.data(), sc, hrow.size() * 8, hipMemcpyDeviceToHost, s));
  if (hist_host) {
    for (int sh = 0; sh < ns; ++sh)
      SSX_HIP(hipMemcpyAsync(hist_host + (size_t)sh * (maxit + 1) * 4,
                             hist + (size_t)sh * (maxit + 1) * 4, (size_t)(maxit + 1) * 4 * 8,
                             hipMemcpyDeviceToHost, s));
  }
  SSX_HIP(hipStreamSynchronize(s));
  if (iters_host) *iters_host = iters;
  int worst = 0;
  for (int sh = 0; sh < ns; ++sh) worst |= (int)hrow[(size_t)sh * SC_N + SC_FLAG];
  if (worst & 2) return fail(SSX_ERR_NONFINITE, "a non-finite PCG scalar appeared");
  if (worst & 1) return fail(SSX_ERR_BREAKDOWN, "PCG breakdown: <g,r> or <p,q> became zero");
  return SSX_OK;
}

}  // namespace

extern "C" {

ssx_status ssx_pcg_solve(ssx_ctx* c, const void* d, double alpha_rel, int32_t maxit,
                         double rtol, int32_t use_precond, void* h_out, double* hist_host,
                         int32_t* iters_host) {
  if (!c || !d || !h_out) return fail(SSX_ERR_ARG, "null argument");
  if (maxit < 0 || maxit > HIST_CAP) return fail(SSX_ERR_ARG, "maxit out of range");
  if (!std::isfinite(alpha_rel) || alpha_rel < 0) return fail(SSX_ERR_ARG, "alpha_rel must be >= 0");
  return run_pcg(c, Pcg::EUCLID, d, alpha_rel, maxit, rtol, use_precond, h_out, hist_host,
                 iters_host);
}

ssx_status ssx_batch_create(int32_t n, ssx_ctx* const* ctxs, ssx_batch** out) {
  if (!out) return fail(SSX_ERR_ARG, "null argument");
  *out = nullptr;
  if (n < 1 || !ctxs) return fail(SSX_ERR_ARG, "a batch needs at least one context");
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(SSX_ERR_ARG, "null context in the batch");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(SSX_ERR_ARG, "a context appears twice in the batch");
    const ssx_ctx* c = ctxs[i];
    const ssx_ctx* c0 = ctxs[0];
    if (c->prob.order != c0->prob.order || c->fdt != c0->fdt || c->vdbl != c0->vdbl)
      return fail(SSX_ERR_ARG, "batch contexts must share the stencil order, field and vector types");
    if (c->stream != c0->stream) return fail(SSX_ERR_ARG, "batch contexts must share one stream");
  }
  ssx_batch* b = new ssx_batch();
  b->ctx.assign(ctxs, ctxs + n);
  b->stream = ctxs[0]->stream;
  b->fdt = ctxs[0]->fdt;
  b->order = ctxs[0]->prob.order;
  b->graphs = ctxs[0]->graphs;
  *out = b;
  return SSX_OK;
}

ssx_status ssx_batch_pcg_solve(ssx_batch* b, const void* const* d, const double* alpha_rel,
                               int32_t maxit, double rtol, int32_t use_precond,
                               void* const* h_out, double* const* hist_host, int32_t* iters_host,
                               int32_t* status_host) {
  if (!b || !d || !alpha_rel || !h_out) return fail(SSX_ERR_ARG, "null argument");
  if (maxit < 0 || maxit > HIST_CAP) return fail(SSX_ERR_ARG, "maxit out of range");
  const int n = (int)b->ctx.size();
  for (int i = 0; i < n; ++i) {
    if (!d[i] || !h_out[i]) return fail(SSX_ERR_ARG, "null data or output in the batch");
    if (!std::isfinite(alpha_rel[i]) || alpha_rel[i] < 0)
      return fail(SSX_ERR_ARG, "alpha_rel must be >= 0");
  }
  int dev = 0;
  SSX_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->active = n;
    b->pending.clear();
  }
  std::vector<ssx_status> st(n, SSX_OK);
  std::vector<std::string> err(n);
  std::vector<std::thread> th;
  th.reserve(n);
  int started = 0;
  for (int i = 0; i < n; ++i) {
    auto member = [&, i] {
      const hipError_t e = hipSetDevice(dev);
      if (e != hipSuccess) {
        st[i] = fail(SSX_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
      } else {
        tl_batch = b;
        st[i] = run_pcg(b->ctx[i], Pcg::EUCLID, d[i], alpha_rel[i], maxit, rtol, use_precond,
                        h_out[i], hist_host ? hist_host[i] : nullptr,
                        iters_host ? iters_host + i : nullptr);
        tl_batch = nullptr;
      }
      if (st[i] != SSX_OK) err[i] = g_err;
      std::lock_guard<std::mutex> lk(b->mu);
      --b->active;
      batch_maybe_flush(b);
    };
    try {
      th.emplace_back(member);
      ++started;
    } catch (...) {
      break;
    }
  }
  if (started < n) {
    // a thread could not be started: the members that run go on without
    // the others (who never arrive at the barrier), and the call fails
    std::lock_guard<std::mutex> lk(b->mu);
    b->active -= n - started;
    batch_maybe_flush(b);
  }
  for (std::thread& t : th) t.join();
  if (started < n)
    return fail(SSX_ERR_OOM, "could not start a host thread for batch member " +
                                 std::to_string(started));
  if (status_host)
    for (int i = 0; i < n; ++i) status_host[i] = st[i];
  for (int i = 0; i < n; ++i)
    if (st[i] != SSX_OK) return fail(st[i], "batch member " + std::to_string(i) + ": " + err[i]);
  return SSX_OK;
}

void ssx_batch_destroy(ssx_batch* b) {
  if (!b) return;
  for (BatchGraphEntry& e : b->graph_cache) (void)hipGraphExecDestroy(e.exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
}

ssx_status ssx_weight_d(ssx_ctx* c, const void* r, void* y) {
  if (!c || !r || !y) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_rslab) return fail(SSX_ERR_ARG, "context has no receiver-side slab (rslab_dz == 0)");
  return do_wd(c, r, y);
}

ssx_status ssx_weight_m(ssx_ctx* c, const void* x, void* y) {
  if (!c || !x || !y) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_rslab) return fail(SSX_ERR_ARG, "context has no receiver-side slab (rslab_dz == 0)");
  return do_wm(c, x, y);
}

ssx_status ssx_normal_w(ssx_ctx* c, double alpha, const void* p, void* q, void* Fp) {
  if (!c || !p || !q) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_rslab) return fail(SSX_ERR_ARG, "context has no receiver-side slab (rslab_dz == 0)");
  if (!std::isfinite(alpha)) return fail(SSX_ERR_ARG, "alpha must be finite");
  return do_normal_w(c, nullptr, alpha * alpha, alpha != 0.0, p, q, Fp ? Fp : c->t2);
}

ssx_status ssx_pcg_solve_w(ssx_ctx* c, const void* d, double alpha, int32_t maxit, double rtol,
                           int32_t use_precond, void* h_out, double* hist_host,
                           int32_t* iters_host) {
  if (!c || !d || !h_out) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_rslab) return fail(SSX_ERR_ARG, "context has no receiver-side slab (rslab_dz == 0)");
  if (maxit < 0 || maxit > HIST_CAP) return fail(SSX_ERR_ARG, "maxit out of range");
  if (!std::isfinite(alpha) || alpha < 0) return fail(SSX_ERR_ARG, "alpha must be >= 0");
  return run_pcg(c, Pcg::WEIGHTED, d, alpha, maxit, rtol, use_precond, h_out, hist_host,
                 iters_host);
}

ssx_status ssx_pcg_solve_v(ssx_ctx* c, const void* d, double alpha_rel, int32_t maxit,
                           double rtol, void* f_out, double* hist_host, int32_t* iters_host) {
  if (!c || !d || !f_out) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_v) return fail(SSX_ERR_ARG, "no normal-velocity rows at the source or receiver depth");
  if (maxit < 0 || maxit > HIST_CAP) return fail(SSX_ERR_ARG, "maxit out of range");
  if (!std::isfinite(alpha_rel) || alpha_rel < 0) return fail(SSX_ERR_ARG, "alpha_rel must be >= 0");
  return run_pcg(c, Pcg::VELOCITY, d, alpha_rel, maxit, rtol, 0, f_out, hist_host, iters_host);
}

ssx_status ssx_fwd_v(ssx_ctx* c, const void* f, void* y) {
  if (!c || !f || !y) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_v) return fail(SSX_ERR_ARG, "no normal-velocity rows at the source or receiver depth");
  return do_fwd_v(c, f, y);
}

ssx_status ssx_adj_v(ssx_ctx* c, const void* r, void* g) {
  if (!c || !r || !g) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_v) return fail(SSX_ERR_ARG, "no normal-velocity rows at the source or receiver depth");
  return do_adj_v(c, r, g, false);
}

ssx_status ssx_tr_inverse(ssx_ctx* c, const void* d, void* h) {
  if (!c || !d || !h) return fail(SSX_ERR_ARG, "null argument");
  if (!c->has_v) return fail(SSX_ERR_ARG, "no normal-velocity rows at the source or receiver depth");
  return do_adj_v(c, d, h, true);
}

ssx_status ssx_block(ssx_ctx* c, int32_t src, int32_t rec, int32_t transpose, const void* x,
                     void* y) {
  if (!c || !x || !y) return fail(SSX_ERR_ARG, "null argument");
  if ((src != 0 && src != 1) || (rec != 0 && rec != 1))
    return fail(SSX_ERR_ARG, "src and rec must be 0 (pressure) or 1 (normal load / velocity)");
  if (src == 0 && rec == 0) return transpose ? do_adj(c, x, y) : do_fwd(c, x, y);
  if (!c->has_v) return fail(SSX_ERR_ARG, "no normal-velocity rows at the source or receiver depth");
  if (src == 1 && rec == 1) return transpose ? do_adj_v(c, x, y, false) : do_fwd_v(c, x, y);
  return do_block(c, src, rec, transpose != 0, x, y);
}

ssx_status ssx_misfit_gradient(ssx_ctx* c, const void* h, const void* d, void* g,
                               double* J_host) {
  if (!c || !h || !d || !g) return fail(SSX_ERR_ARG, "null argument");
  if (c->fdt != Dt::F64 && c->fdt != Dt::F32)
    return fail(SSX_ERR_ARG, "the misfit gradient needs F64 or F32 fields");
  return do_gradient(c, h, d, g, J_host);
}

ssx_status ssx_lambda(ssx_ctx* c, int32_t side, int32_t transpose, const void* x, void* y) {
  if (!c || !x || !y) return fail(SSX_ERR_ARG, "null argument");
  if (side != 0 && side != 1) return fail(SSX_ERR_ARG, "side must be 0 (source) or 1 (receiver)");
  if (side == 1 && !c->has_rslab)
    return fail(SSX_ERR_ARG, "context has no receiver-side slab (rslab_dz == 0)");
  return do_lambda(c, side, transpose != 0, x, y);
}

ssx_status ssx_set_option(ssx_ctx* c, int option, int value) {
  if (!c) return fail(SSX_ERR_ARG, "null context");
  switch (option) {
    case SSX_OPT_GRAPHS:
      c->graphs = value != 0;
      return SSX_OK;
    case SSX_OPT_STEP_KERNEL:
      if (value != 0 && value != 1) return fail(SSX_ERR_ARG, "step kernel must be 0 or 1");
      c->fused = value == 1;
      return SSX_OK;
    case SSX_OPT_TILE_Z:
    case SSX_OPT_TILE_Z_SLAB:
      if (value != 0 && value != 8 && value != 16 && value != 32)
        return fail(SSX_ERR_ARG, "tile height must be 0, 8, 16 or 32");
      if (value == 32 && c->fdt == Dt::F64)
        return fail(SSX_ERR_ARG, "tile height 32 is not available for F64 fields");
      if (option == SSX_OPT_TILE_Z) c->tile_z_full = value;
      c->tile_z_slab = value;
      return SSX_OK;
    case SSX_OPT_STEPS_PER_LAUNCH:
      if (value != 1 && value != 2 && value != 4 && value != 8)
        return fail(SSX_ERR_ARG, "steps per launch must be 1, 2, 4 or 8");
      if (value > 1 && !multi_ok(c, c->full.host.NZ, value, multi_strip(c, true, value)))
        return SSX_ERR_ARG;
      c->spl_full = value;
      return SSX_OK;
    case SSX_OPT_STEPS_PER_LAUNCH_SLAB:
      if (value != 1 && value != 2 && value != 4 && value != 8)
        return fail(SSX_ERR_ARG, "steps per launch must be 1, 2, 4 or 8");
      if (value > 1) {
        const int wr = multi_strip(c, false, value);
        if (!multi_ok(c, c->slab.host.NZ, value, wr)) return SSX_ERR_ARG;
        if (c->has_rslab && !multi_ok(c, c->rslab.host.NZ, value, wr)) return SSX_ERR_ARG;
      }
      c->spl_slab = value;
      return SSX_OK;
    case SSX_OPT_SLAB_STRIP:
    case SSX_OPT_STRIP:
      if (value != 0 && value != 64 && value != 128)
        return fail(SSX_ERR_ARG, "strip width must be 0, 64 or 128");
      if (option == SSX_OPT_STRIP) {
        const int old = c->strip_full;
        c->strip_full = value;
        if (c->spl_full > 1 &&
            !multi_ok(c, c->full.host.NZ, c->spl_full, multi_strip(c, true, c->spl_full))) {
          c->strip_full = old;
          return SSX_ERR_ARG;
        }
      } else {
        const int old = c->slab_strip;
        c->slab_strip = value;
        const int wr = multi_strip(c, false, c->spl_slab);
        if (c->spl_slab > 1 && (!multi_ok(c, c->slab.host.NZ, c->spl_slab, wr) ||
                                (c->has_rslab && !multi_ok(c, c->rslab.host.NZ, c->spl_slab, wr)))) {
          c->slab_strip = old;
          return SSX_ERR_ARG;
        }
      }
      return SSX_OK;
    case SSX_OPT_SHOT_GROUP:
    case SSX_OPT_SHOT_GROUP_SLAB:
      if (value < 0) return fail(SSX_ERR_ARG, "shots per launch must be >= 0");
      if (option == SSX_OPT_SHOT_GROUP) c->group_full = value;
      c->group_slab = value;
      return SSX_OK;
    case SSX_OPT_TILE_LOOP:
      if (value != 0 && value != 1 && value < 8)
        return fail(SSX_ERR_ARG, "tile loop must be 0, 1 or at least 8");
      if (value != 0 && c->vrho)
        return fail(SSX_ERR_ARG, "the tile loop takes constant density only");
      c->loop_full = value;
      return SSX_OK;
    case SSX_OPT_OVERLAP:
      if (value != 0 && value != 1) return fail(SSX_ERR_ARG, "overlap must be 0 or 1");
      c->overlap = value == 1;
      return SSX_OK;
  }
  return fail(SSX_ERR_ARG, "unknown option");
}

const char* ssx_last_error(void) { return g_err.c_str(); }

const char* ssx_step_kernel_name(ssx_ctx* c) {
  if (c && !c->fused) return "k_vel + k_pres";
  if (c && c->spl_full > 1) return "k_slab";
  return "k_step";
}

ssx_status ssx_launch_shape(ssx_ctx* c, int32_t* shape) {
  if (!c || !shape) return fail(SSX_ERR_ARG, "null argument");
  shape[0] = c->fused ? (c->tile_z_full ? c->tile_z_full : default_tile_z(c, c->full)) : 0;
  shape[1] = c->fused ? c->spl_full : 1;
  shape[2] = shot_group(c, c->full);
  shape[3] = (c->fused && c->spl_full == 1) ? c->loop_full : 0;
  return SSX_OK;
}

int64_t ssx_cells_per_launch(ssx_ctx* c) {
  if (!c) return 0;
  return (int64_t)c->full.host.NZ * c->full.host.NX * shot_group(c, c->full);
}

}  // extern "C"
