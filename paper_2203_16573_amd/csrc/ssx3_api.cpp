// Host side of the 3D entry points (ssx3_*): problem and model checks, the
// padded model and absorbing-layer factors of the full grid and of the thin
// slab, the context's device buffers, and the time loops and compositions
// of F, F^T, the penalty, M^-1 = D W^-1 D and Algorithm 1 (kernels in
// ssx3.hip).
#include "ssx.h"
#include "ssx3_internal.h"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

namespace ssx {
void set_last_error(const std::string& msg);  // ssx_api.cpp: ssx_last_error's text
}

using ssx3::Dims3;
using ssx3::Plane3;

namespace {

// One padded grid on the device: the fields, ck, layer factors.
struct Grid3Dev {
  Dims3 d{};
  void* fields = nullptr;
  void* ck = nullptr;
  void* fac = nullptr;
  long long cells() const { return (long long)d.NZ * d.NY * d.NX; }
};

}  // namespace

struct ssx3_ctx {
  ssx3_problem prob{};
  bool f64 = false;
  size_t esz = 0;
  hipStream_t stream = nullptr;
  double cb = 0.0;
  void* buf = nullptr;  // every device array of the context
  Grid3Dev full{}, slab{};
  Plane3 src{}, rec{};        // full grid: pressure source, receivers
  Plane3 fpl{}, dpl{}, dvl{};  // slab: normal load at z_s, datum p and v_z
  double* dist = nullptr;      // [ns] lateral distance from (x_s, y_s), FP64
  double* partial = nullptr;   // [256] dot partials
  double* dot_out = nullptr;   // [1]
  // trace work vectors, field type: [nt][ns] t1, t2, Ps, Vs, r, g, p, q;
  // [nt][nr] Fp, e
  void *t1 = nullptr, *t2 = nullptr, *Ps = nullptr, *Vs = nullptr;
  void *r = nullptr, *g = nullptr, *p = nullptr, *q = nullptr, *Fp = nullptr, *e = nullptr;
};

namespace {

ssx_status fail3(ssx_status s, const std::string& msg) {
  ssx::set_last_error(msg);
  return s;
}

#define S3_HIP(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      ssx::set_last_error(std::string(#expr) + ": " + hipGetErrorString(e_));    \
      return SSX_ERR_HIP;                                                        \
    }                                                                            \
  } while (0)

#define S3_TRY(expr)              \
  do {                            \
    ssx_status s_ = (expr);       \
    if (s_ != SSX_OK) return s_;  \
  } while (0)

// sum of |c_m| of the staggered first-derivative weights
double weight_sum(int order) {
  return order == 4 ? 9.0 / 8.0 + 1.0 / 24.0
                    : 1225.0 / 1024.0 + 245.0 / 3072.0 + 49.0 / 5120.0 + 5.0 / 7168.0;
}

bool on_node(double pos, double h, int n, int count) {
  const double j = pos / h;
  if (!(std::fabs(j - std::round(j)) <= 1e-9)) return false;
  const long long j0 = std::llround(j);
  return j0 >= 0 && j0 + count - 1 <= n - 1;
}

// rows and weights of a plane at depth z (metres from the first physical
// node) of a grid of nz physical planes and L absorbing cells: on pressure
// nodes, or (vz) on v_z half nodes, plane i at depth (i - L + 1/2) h
bool plane_rows(double z, double h, int L, int nz, bool vz, Plane3* pl) {
  const double u = L + z / h - (vz ? 0.5 : 0.0);
  const int i0 = (int)std::floor(u + 1e-12);
  double w1 = u - i0;
  if (std::fabs(w1) < 1e-12) w1 = 0.0;
  pl->r0 = i0;
  pl->w0 = 1.0 - w1;
  pl->r1 = w1 == 0.0 ? -1 : i0 + 1;
  pl->w1 = w1;
  const int lo = L, hi = L + nz - (vz ? 2 : 1);
  return i0 >= lo && i0 <= hi && (pl->r1 < 0 || pl->r1 <= hi);
}

// the thin slab's physical planes [i_lo, i_hi] of the full model (clamped
// into it when they reach past its top or bottom): from min(i, i + dz) - k
// to max(i, i + dz) + k, i the plane at or above z_s, one more below when
// z_s falls between planes, k = order / 2
void slab_planes(const ssx3_problem& p, int* i_lo, int* i_hi) {
  const int k = p.order / 2, dz = p.slab_dz;
  const int i_s = (int)std::floor(p.z_src / p.h + 1e-12);
  *i_lo = std::min(i_s, i_s + dz) - k;
  *i_hi = std::max(i_s, i_s + dz) + k + (p.z_src / p.h - i_s > 1e-12 ? 1 : 0);
}

Plane3 lateral(Plane3 pl, int L, double x0, int nx, double y0, int ny, double h) {
  pl.x0 = L + (int)std::llround(x0 / h);
  pl.nx = nx;
  pl.y0 = L + (int)std::llround(y0 / h);
  pl.ny = ny;
  return pl;
}

ssx_status check3(const ssx3_problem* p) {
  if (!p) return fail3(SSX_ERR_ARG, "problem is NULL");
  if (p->order != 4 && p->order != 8) return fail3(SSX_ERR_ARG, "order must be 4 or 8");
  if (p->nz < p->order + 1 || p->ny < p->order + 1 || p->nx < p->order + 1)
    return fail3(SSX_ERR_ARG, "grid smaller than order + 1 nodes on an axis");
  if (p->npml < 0) return fail3(SSX_ERR_ARG, "npml must be >= 0");
  if (!(p->h > 0.0) || !(p->dt > 0.0) || p->nt < 1)
    return fail3(SSX_ERR_ARG, "h, dt and nt must be positive");
  if (!(p->pml_R > 0.0 && p->pml_R < 1.0)) return fail3(SSX_ERR_ARG, "pml_R must lie in (0, 1)");
  if (p->field_dtype != SSX_F64 && p->field_dtype != SSX_F32)
    return fail3(SSX_ERR_ARG, "3D fields are F64 or F32");
  if (p->nsx < 1 || p->nsy < 1 || p->nrx < 1 || p->nry < 1)
    return fail3(SSX_ERR_ARG, "planes need at least one trace");
  if (!on_node(p->x_src0, p->h, p->nx, p->nsx) || !on_node(p->y_src0, p->h, p->ny, p->nsy) ||
      !on_node(p->x_rec0, p->h, p->nx, p->nrx) || !on_node(p->y_rec0, p->h, p->ny, p->nry))
    return fail3(SSX_ERR_ARG, "plane traces must lie on grid nodes inside the physical grid");
  Plane3 t{};
  if (!plane_rows(p->z_src, p->h, p->npml, p->nz, false, &t) ||
      !plane_rows(p->z_rec, p->h, p->npml, p->nz, false, &t))
    return fail3(SSX_ERR_ARG, "plane depth outside the physical grid");
  if (p->slab_dz == 0) return fail3(SSX_ERR_ARG, "slab_dz must be nonzero");
  if (!std::isfinite(p->x_s) || !std::isfinite(p->y_s))
    return fail3(SSX_ERR_ARG, "x_s and y_s must be finite");
  int i_lo, i_hi;
  slab_planes(*p, &i_lo, &i_hi);
  if (i_hi - i_lo + 1 > 4096) return fail3(SSX_ERR_ARG, "slab_dz too large");
  const long long NZ = p->nz + 2LL * p->npml, NY = p->ny + 2LL * p->npml,
                  NX = p->nx + 2LL * p->npml;
  if (NZ > 65535 || NY * NX > (1LL << 31) || NZ * NY * NX > (1LL << 40))
    return fail3(SSX_ERR_ARG, "grid too large");
  return SSX_OK;
}

// c_max of kappa over the physical planes [z0, z1] (all rows and columns)
double cmax_of(const ssx3_problem& p, const double* kappa, double rho, int z0, int z1) {
  double kmax = 0.0;
  for (long long i = (long long)z0 * p.ny * p.nx; i < (long long)(z1 + 1) * p.ny * p.nx; ++i)
    kmax = std::max(kmax, kappa[i]);
  return std::sqrt(kmax / rho);
}

ssx_status check_model3(const ssx3_problem& p, const double* kappa, double rho, double* cmax) {
  if (!(std::isfinite(rho) && rho > 0.0)) return fail3(SSX_ERR_ARG, "rho must be finite and > 0");
  const long long n = (long long)p.nz * p.ny * p.nx;
  for (long long i = 0; i < n; ++i)
    if (!(std::isfinite(kappa[i]) && kappa[i] > 0.0))
      return fail3(SSX_ERR_ARG, "kappa must be finite and > 0");
  *cmax = cmax_of(p, kappa, rho, 0, p.nz - 1);
  // leapfrog stability on the 3D staggered grid
  if (*cmax * p.dt / p.h > 1.0 / (std::sqrt(3.0) * weight_sum(p.order)))
    return fail3(SSX_ERR_CFL, "dt above the 3D stability bound");
  return SSX_OK;
}

Dims3 dims_of(const ssx3_problem& p, int nz) {
  return {nz + 2 * p.npml, p.ny + 2 * p.npml, p.nx + 2 * p.npml, p.npml};
}

long long grid_elems(const Dims3& d) {
  return (ssx3::NFIELDS3 + 1LL) * d.NZ * d.NY * d.NX + 4LL * (d.NZ + d.NY + d.NX);
}

// bytes of every device array of a context
size_t bytes_of(const ssx3_problem& p) {
  int i_lo, i_hi;
  slab_planes(p, &i_lo, &i_hi);
  const size_t esz = p.field_dtype == SSX_F64 ? 8 : 4;
  const long long ns = (long long)p.nsx * p.nsy * p.nt, nr = (long long)p.nrx * p.nry * p.nt;
  const long long elems = grid_elems(dims_of(p, p.nz)) + grid_elems(dims_of(p, i_hi - i_lo + 1)) +
                          8 * ns + 2 * nr;
  return (size_t)elems * esz + (size_t)(p.nsx * (long long)p.nsy + 256 + 1) * 8 + 256;
}

// ck and layer factors of a grid whose physical planes are the full model's
// planes rows[0..nzg) (rows outside the model clamped into it)
template <typename T>
void fill_coefs(const ssx3_problem& p, const Dims3& d, const std::vector<int>& rows,
                const double* kappa, double cmax, std::vector<T>& ck, std::vector<T>& fac) {
  const int L = p.npml, nzg = (int)rows.size();
  ck.resize((size_t)d.NZ * d.NY * d.NX);
  // the model extended into the layer by the nearest physical value
  for (int z = 0; z < d.NZ; ++z) {
    const int iz = rows[std::min(std::max(z - L, 0), nzg - 1)];
    for (int y = 0; y < d.NY; ++y) {
      const int iy = std::min(std::max(y - L, 0), p.ny - 1);
      for (int x = 0; x < d.NX; ++x) {
        const int ix = std::min(std::max(x - L, 0), p.nx - 1);
        const double k = kappa[((size_t)iz * p.ny + iy) * p.nx + ix];
        ck[((size_t)z * d.NY + y) * d.NX + x] = T(p.dt * k / p.h);
      }
    }
  }
  // split-field layer: sigma(d) = sigma_max (d / (L h))^2 with d the depth
  // into the layer, sigma_max = 3 c_max ln(1/R) / (2 L h); a field damped by
  // sigma advances with a = (1 - sigma dt/2) / (1 + sigma dt/2) on its old
  // value and b = 1 / (1 + sigma dt/2) on its update
  const double smax = L > 0 ? 3.0 * cmax * std::log(1.0 / p.pml_R) / (2.0 * L * p.h) : 0.0;
  auto sigma = [&](double pos, int n) {
    const double dd = std::max(std::max(L - pos, pos - (L + n - 1)), 0.0);
    return L > 0 ? smax * (dd / L) * (dd / L) : 0.0;
  };
  fac.clear();
  const int Ns[3] = {d.NZ, d.NY, d.NX}, ns[3] = {nzg, p.ny, p.nx};
  for (int a = 0; a < 3; ++a) {
    std::vector<T> an(Ns[a]), bn(Ns[a]), ah(Ns[a]), bh(Ns[a]);
    for (int i = 0; i < Ns[a]; ++i) {
      const double qn = 0.5 * sigma(i, ns[a]) * p.dt, qh = 0.5 * sigma(i + 0.5, ns[a]) * p.dt;
      an[i] = T((1.0 - qn) / (1.0 + qn));
      bn[i] = T(1.0 / (1.0 + qn));
      ah[i] = T((1.0 - qh) / (1.0 + qh));
      bh[i] = T(1.0 / (1.0 + qh));
    }
    fac.insert(fac.end(), an.begin(), an.end());
    fac.insert(fac.end(), bn.begin(), bn.end());
    fac.insert(fac.end(), ah.begin(), ah.end());
    fac.insert(fac.end(), bh.begin(), bh.end());
  }
}

template <typename T>
hipError_t upload_grid(const ssx3_problem& p, const Grid3Dev& g, const std::vector<int>& rows,
                       const double* kappa, double cmax) {
  std::vector<T> ck, fac;
  fill_coefs<T>(p, g.d, rows, kappa, cmax, ck, fac);
  hipError_t e = hipMemcpy(g.ck, ck.data(), ck.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(g.fac, fac.data(), fac.size() * sizeof(T), hipMemcpyHostToDevice);
}

const char* at(const void* base, long long elems, size_t esz) {
  return static_cast<const char*>(base) + elems * (long long)esz;
}
char* at(void* base, long long elems, size_t esz) {
  return static_cast<char*>(base) + elems * (long long)esz;
}

long long nsv(const ssx3_problem& p) { return (long long)p.nsx * p.nsy; }
long long nrv(const ssx3_problem& p) { return (long long)p.nrx * p.nry; }

const Plane3 kNone{0, -1, 0.0, 0.0, 0, 0, 0, 0};

// Forward sweep on grid g: pressure source (hp, h) and normal load (fp, f)
// (null: none); records the pressure on rp into P and v_z on vp into V
// (null: not recorded); traces [nt][n] of each plane.
ssx_status sweep_fwd(ssx3_ctx* c, const Grid3Dev& g, const Plane3& hp, const void* h,
                     const Plane3& fp, const void* f, const Plane3& rp, void* P,
                     const Plane3& vp, void* V) {
  const ssx3_problem& p = c->prob;
  const long long nh = (long long)hp.nx * hp.ny, nf = (long long)fp.nx * fp.ny;
  const long long np = (long long)rp.nx * rp.ny, nv = (long long)vp.nx * vp.ny;
  S3_HIP(hipMemsetAsync(g.fields, 0, ssx3::NFIELDS3 * g.cells() * c->esz, c->stream));
  for (int t = 0; t < p.nt; ++t) {
    S3_HIP(ssx3::launch3_step(c->f64, p.order, false, g.fields, g.d, g.fac, g.ck, c->cb, hp,
                              h ? at(h, t * nh, c->esz) : nullptr, fp,
                              f ? at(f, t * nf, c->esz) : nullptr, c->stream));
    if (P)
      S3_HIP(ssx3::launch3_gather(c->f64, 0, g.fields, g.d, rp, g.fac, g.ck, c->cb,
                                  at(P, t * np, c->esz), c->stream));
    if (V)
      S3_HIP(ssx3::launch3_gather(c->f64, 2, g.fields, g.d, vp, g.fac, g.ck, c->cb,
                                  at(V, t * nv, c->esz), c->stream));
  }
  return SSX_OK;
}

// Transposed sweep on grid g: the pressure recording's adjoint input a on
// rp and the v_z recording's b on vp (null: none); outputs the
// pressure-source slot on hp into H and the normal-load slot on fp into F
// (null: not read).
ssx_status sweep_adj(ssx3_ctx* c, const Grid3Dev& g, const Plane3& rp, const void* a,
                     const Plane3& vp, const void* b, const Plane3& hp, void* H,
                     const Plane3& fp, void* F) {
  const ssx3_problem& p = c->prob;
  const long long nh = (long long)hp.nx * hp.ny, nf = (long long)fp.nx * fp.ny;
  const long long np = (long long)rp.nx * rp.ny, nv = (long long)vp.nx * vp.ny;
  S3_HIP(hipMemsetAsync(g.fields, 0, ssx3::NFIELDS3 * g.cells() * c->esz, c->stream));
  if (a)
    S3_HIP(ssx3::launch3_spread(c->f64, g.fields, g.d, rp, g.fac, g.ck,
                                at(a, (p.nt - 1) * np, c->esz), c->stream));
  for (int t = p.nt - 1; t >= 0; --t) {
    if (H)
      S3_HIP(ssx3::launch3_gather(c->f64, 1, g.fields, g.d, hp, g.fac, g.ck, c->cb,
                                  at(H, t * nh, c->esz), c->stream));
    // the velocity adjoints (with this step's v_z recording), then the
    // pressure adjoints (with the next-lower step's pressure recording);
    // the latter leave v_z's adjoint as the former wrote it, so the
    // normal-load slot is read after both
    S3_HIP(ssx3::launch3_step(c->f64, p.order, true, g.fields, g.d, g.fac, g.ck, c->cb, rp,
                              (a && t >= 1) ? at(a, (t - 1) * np, c->esz) : nullptr, vp,
                              b ? at(b, t * nv, c->esz) : nullptr, c->stream));
    if (F)
      S3_HIP(ssx3::launch3_gather(c->f64, 3, g.fields, g.d, fp, g.fac, g.ck, c->cb,
                                  at(F, t * nf, c->esz), c->stream));
  }
  return SSX_OK;
}

}  // namespace

extern "C" {

ssx_status ssx3_validate(const ssx3_problem* prob, const double* kappa_host, double rho) {
  const ssx_status s = check3(prob);
  if (s != SSX_OK || !kappa_host) return s;
  double cmax;
  return check_model3(*prob, kappa_host, rho, &cmax);
}

size_t ssx3_footprint(const ssx3_problem* prob) {
  if (check3(prob) != SSX_OK) return 0;
  return bytes_of(*prob);
}

ssx_status ssx3_create(const ssx3_problem* prob, const double* kappa_host, double rho,
                       void* stream, ssx3_ctx** out) {
  if (!out) return fail3(SSX_ERR_ARG, "out is NULL");
  *out = nullptr;
  S3_TRY(check3(prob));
  if (!kappa_host) return fail3(SSX_ERR_ARG, "kappa_host is required");
  double cmax;
  S3_TRY(check_model3(*prob, kappa_host, rho, &cmax));
  ssx3_ctx* c = new ssx3_ctx();
  c->prob = *prob;
  const ssx3_problem& p = c->prob;
  c->f64 = p.field_dtype == SSX_F64;
  c->esz = c->f64 ? 8 : 4;
  c->stream = static_cast<hipStream_t>(stream);
  c->cb = p.dt / (rho * p.h);
  const int L = p.npml;
  // full grid and its planes
  c->full.d = dims_of(p, p.nz);
  plane_rows(p.z_src, p.h, L, p.nz, false, &c->src);
  plane_rows(p.z_rec, p.h, L, p.nz, false, &c->rec);
  c->src = lateral(c->src, L, p.x_src0, p.nsx, p.y_src0, p.nsy, p.h);
  c->rec = lateral(c->rec, L, p.x_rec0, p.nrx, p.y_rec0, p.nry, p.h);
  // thin slab around z_s and its planes: the normal load at z_s (v_z
  // nodes), the datum slab_dz cells away on p and on v_z nodes
  int i_lo, i_hi;
  slab_planes(p, &i_lo, &i_hi);
  const int nzs = i_hi - i_lo + 1;
  c->slab.d = dims_of(p, nzs);
  const double zl = p.z_src - i_lo * p.h, zd = zl + p.slab_dz * p.h;
  if (!plane_rows(zl, p.h, L, nzs, true, &c->fpl) || !plane_rows(zd, p.h, L, nzs, false, &c->dpl) ||
      !plane_rows(zd, p.h, L, nzs, true, &c->dvl)) {
    delete c;
    return fail3(SSX_ERR_ARG, "thin-slab planes outside the slab");
  }
  c->fpl = lateral(c->fpl, L, p.x_src0, p.nsx, p.y_src0, p.nsy, p.h);
  c->dpl = lateral(c->dpl, L, p.x_src0, p.nsx, p.y_src0, p.nsy, p.h);
  c->dvl = lateral(c->dvl, L, p.x_src0, p.nsx, p.y_src0, p.nsy, p.h);
  // one device buffer: both grids, the trace work vectors, FP64 scalars
  if (hipMalloc(&c->buf, bytes_of(p)) != hipSuccess) {
    delete c;
    (void)hipGetLastError();
    return fail3(SSX_ERR_OOM, "device allocation failed");
  }
  char* b = static_cast<char*>(c->buf);
  auto carve = [&](long long elems) {
    void* r = b;
    b += elems * (long long)c->esz;
    return r;
  };
  for (Grid3Dev* g : {&c->full, &c->slab}) {
    const long long n = g->cells();
    g->fields = carve(ssx3::NFIELDS3 * n);
    g->ck = carve(n);
    g->fac = carve(4LL * (g->d.NZ + g->d.NY + g->d.NX));
  }
  const long long ns = nsv(p) * p.nt, nr = nrv(p) * p.nt;
  void** sv[] = {&c->t1, &c->t2, &c->Ps, &c->Vs, &c->r, &c->g, &c->p, &c->q};
  for (void** v : sv) *v = carve(ns);
  c->Fp = carve(nr);
  c->e = carve(nr);
  b = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(b) + 255) & ~uintptr_t(255));
  c->dist = reinterpret_cast<double*>(b);
  c->partial = c->dist + nsv(p);
  c->dot_out = c->partial + 256;
  // coefficients
  std::vector<int> rows_full(p.nz), rows_slab(nzs);
  for (int i = 0; i < p.nz; ++i) rows_full[i] = i;
  for (int i = 0; i < nzs; ++i) rows_slab[i] = std::min(std::max(i_lo + i, 0), p.nz - 1);
  const double cmax_s = cmax_of(p, kappa_host, rho, std::max(i_lo, 0), std::min(i_hi, p.nz - 1));
  std::vector<double> dist(nsv(p));
  for (int yb = 0; yb < p.nsy; ++yb)
    for (int xa = 0; xa < p.nsx; ++xa) {
      const double dx = p.x_src0 + p.h * xa - p.x_s, dy = p.y_src0 + p.h * yb - p.y_s;
      dist[(size_t)yb * p.nsx + xa] = std::sqrt(dx * dx + dy * dy);
    }
  hipError_t e1 = c->f64 ? upload_grid<double>(p, c->full, rows_full, kappa_host, cmax)
                         : upload_grid<float>(p, c->full, rows_full, kappa_host, cmax);
  if (e1 == hipSuccess)
    e1 = c->f64 ? upload_grid<double>(p, c->slab, rows_slab, kappa_host, cmax_s)
                : upload_grid<float>(p, c->slab, rows_slab, kappa_host, cmax_s);
  if (e1 == hipSuccess)
    e1 = hipMemcpy(c->dist, dist.data(), dist.size() * 8, hipMemcpyHostToDevice);
  if (e1 != hipSuccess) {
    (void)hipFree(c->buf);
    delete c;
    return fail3(SSX_ERR_HIP, std::string("coefficient upload: ") + hipGetErrorString(e1));
  }
  *out = c;
  return SSX_OK;
}

ssx_status ssx3_fwd(ssx3_ctx* c, const void* h, void* d) {
  if (!c || !h || !d) return fail3(SSX_ERR_ARG, "null argument");
  return sweep_fwd(c, c->full, c->src, h, kNone, nullptr, c->rec, d, kNone, nullptr);
}

ssx_status ssx3_adj(ssx3_ctx* c, const void* r, void* g) {
  if (!c || !r || !g) return fail3(SSX_ERR_ARG, "null argument");
  return sweep_adj(c, c->full, c->rec, r, kNone, nullptr, c->src, g, kNone, nullptr);
}

ssx_status ssx3_penalty(ssx3_ctx* c, int op, double a, const void* x, void* y) {
  if (!c || !x || !y) return fail3(SSX_ERR_ARG, "null argument");
  if (op < 0 || op > 2) return fail3(SSX_ERR_ARG, "unknown penalty operator");
  const ssx3_problem& p = c->prob;
  S3_HIP(ssx3::launch3_diag(c->f64, op, a, 1.0, c->dist, x, y, nsv(p) * p.nt, (int)nsv(p),
                            c->stream));
  return SSX_OK;
}

namespace {
// g = M^-1 r = D s X^T J X D r on the thin slab
ssx_status precond3(ssx3_ctx* c, double alpha_hat, const void* r, void* g) {
  const ssx3_problem& p = c->prob;
  const long long n = nsv(p) * p.nt;
  S3_HIP(ssx3::launch3_diag(c->f64, 2, alpha_hat, 1.0, c->dist, r, c->t1, n, (int)nsv(p),
                            c->stream));
  // X: normal load on z_s, datum pressure and v_z recorded
  S3_TRY(sweep_fwd(c, c->slab, kNone, nullptr, c->fpl, c->t1, c->dpl, c->Ps, c->dvl, c->Vs));
  // X^T J: the v_z record in the pressure slot, the pressure record in the
  // v_z slot; read from the normal-load slot
  S3_TRY(sweep_adj(c, c->slab, c->dpl, c->Vs, c->dvl, c->Ps, kNone, nullptr, c->fpl, c->t2));
  const double s = c->prob.slab_dz > 0 ? 4.0 : -4.0;
  S3_HIP(ssx3::launch3_diag(c->f64, 2, alpha_hat, s, c->dist, c->t2, g, n, (int)nsv(p),
                            c->stream));
  return SSX_OK;
}

ssx_status dot3(ssx3_ctx* c, const void* x, const void* y, long long n, double* out) {
  S3_HIP(ssx3::launch3_dot(c->f64, x, y, n, c->partial, c->dot_out, c->stream));
  S3_HIP(hipMemcpyAsync(out, c->dot_out, 8, hipMemcpyDeviceToHost, c->stream));
  S3_HIP(hipStreamSynchronize(c->stream));
  return SSX_OK;
}

ssx_status copy3(ssx3_ctx* c, void* dst, const void* src, long long n) {
  S3_HIP(hipMemcpyAsync(dst, src, n * c->esz, hipMemcpyDeviceToDevice, c->stream));
  return SSX_OK;
}
}  // namespace

ssx_status ssx3_precond(ssx3_ctx* c, double alpha_hat, const void* r, void* g) {
  if (!c || !r || !g) return fail3(SSX_ERR_ARG, "null argument");
  if (!(alpha_hat >= 0.0)) return fail3(SSX_ERR_ARG, "alpha_hat must be >= 0");
  return precond3(c, alpha_hat, r, g);
}

ssx_status ssx3_pcg_solve(ssx3_ctx* c, const void* d, double alpha_rel, int32_t maxit,
                          int32_t use_precond, void* h_out, double* hist_host,
                          int32_t* iters_host) {
  if (!c || !d || !h_out) return fail3(SSX_ERR_ARG, "null argument");
  if (maxit < 0 || maxit > 4096) return fail3(SSX_ERR_ARG, "maxit out of range");
  if (!(alpha_rel >= 0.0)) return fail3(SSX_ERR_ARG, "alpha_rel must be >= 0");
  const ssx3_problem& p = c->prob;
  const long long n = nsv(p) * p.nt, ne = nrv(p) * p.nt;
  hipStream_t s = c->stream;
  // b = F^T d (in r), alpha = alpha_rel ||b|| / ||d||
  S3_TRY(ssx3_adj(c, d, c->r));
  double dd, bb;
  S3_TRY(dot3(c, d, d, ne, &dd));
  S3_TRY(dot3(c, c->r, c->r, n, &bb));
  if (!(dd > 0.0)) return fail3(SSX_ERR_ARG, "the data are zero");
  const double alpha = alpha_rel * std::sqrt(bb) / std::sqrt(dd), a2 = alpha * alpha;
  auto apply_M = [&](const void* r, void* g) -> ssx_status {
    if (use_precond) return precond3(c, alpha_rel, r, g);
    return copy3(c, g, r, n);
  };
  // q = N p = F^T F p + alpha^2 A^T A p, Fp = F p
  auto apply_N = [&]() -> ssx_status {
    S3_TRY(ssx3_fwd(c, c->p, c->Fp));
    S3_TRY(ssx3_adj(c, c->Fp, c->q));
    S3_HIP(ssx3::launch3_diag(c->f64, 1, 0.0, 1.0, c->dist, c->p, c->t1, n, (int)nsv(p), s));
    S3_HIP(ssx3::launch3_axpy(c->f64, c->q, c->q, a2, c->t1, n, s));
    return SSX_OK;
  };
  S3_HIP(hipMemsetAsync(h_out, 0, n * c->esz, s));
  S3_HIP(ssx3::launch3_axpy(c->f64, c->e, d, -2.0, d, ne, s));  // e_0 = F h_0 - d = -d
  S3_TRY(apply_M(c->r, c->g));
  S3_TRY(copy3(c, c->p, c->g, n));
  if (maxit > 0) S3_TRY(apply_N());
  double gr, rr, gg, ee;
  S3_TRY(dot3(c, c->g, c->r, n, &gr));
  auto record = [&](int k) -> ssx_status {
    S3_TRY(dot3(c, c->r, c->r, n, &rr));
    S3_TRY(dot3(c, c->g, c->g, n, &gg));
    S3_TRY(dot3(c, c->e, c->e, ne, &ee));
    if (hist_host) {
      double* row = hist_host + 4 * (size_t)k;
      row[0] = std::sqrt(rr);
      row[1] = std::sqrt(gg);
      row[2] = gr;
      row[3] = std::sqrt(ee);
    }
    return SSX_OK;
  };
  S3_TRY(record(0));
  int iters = 0;
  for (int k = 0; k < maxit; ++k) {
    double pq;
    S3_TRY(dot3(c, c->p, c->q, n, &pq));
    if (!(pq != 0.0) || !(gr != 0.0) || !std::isfinite(pq) || !std::isfinite(gr)) {
      if (iters_host) *iters_host = iters;
      return fail3(std::isfinite(pq) && std::isfinite(gr) ? SSX_ERR_BREAKDOWN : SSX_ERR_NONFINITE,
                   "PCG breakdown: <g,r> or <p,q> became zero or non-finite");
    }
    const double a = gr / pq;
    S3_HIP(ssx3::launch3_axpy(c->f64, h_out, h_out, a, c->p, n, s));
    S3_HIP(ssx3::launch3_axpy(c->f64, c->r, c->r, -a, c->q, n, s));
    S3_HIP(ssx3::launch3_axpy(c->f64, c->e, c->e, a, c->Fp, ne, s));
    S3_TRY(apply_M(c->r, c->g));
    double gr_new;
    S3_TRY(dot3(c, c->g, c->r, n, &gr_new));
    const double beta = gr_new / gr;
    S3_HIP(ssx3::launch3_axpy(c->f64, c->p, c->g, beta, c->p, n, s));
    gr = gr_new;
    S3_TRY(record(k + 1));
    iters = k + 1;
    if (k < maxit - 1) S3_TRY(apply_N());
  }
  S3_HIP(hipStreamSynchronize(s));
  if (iters_host) *iters_host = iters;
  return SSX_OK;
}

void ssx3_destroy(ssx3_ctx* c) {
  if (!c) return;
  if (c->buf) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->buf);
  }
  delete c;
}

}  // extern "C"
