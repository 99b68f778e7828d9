// Host side of the 3D entry points (ssx3_*): problem and model checks, the
// padded model and absorbing-layer factors, the context's device buffer,
// and the time loops of F and its transpose (kernels in ssx3.hip).
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

struct ssx3_ctx {
  ssx3_problem prob{};
  Dims3 d{};
  bool f64 = false;
  size_t esz = 0;
  hipStream_t stream = nullptr;
  void* buf = nullptr;     // fields (7 N), ck (N), layer factors (4 (NZ + NY + NX))
  void* fields = nullptr;
  void* ck = nullptr;
  void* fac = nullptr;
  double cb = 0.0;
  Plane3 src{}, rec{};
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

// rows and weights of a plane at physical depth z on pressure nodes
bool plane_rows(const ssx3_problem& p, double z, Plane3* pl) {
  const double u = p.npml + z / p.h;
  const int i0 = (int)std::floor(u + 1e-12);
  double w1 = u - i0;
  if (std::fabs(w1) < 1e-12) w1 = 0.0;
  pl->r0 = i0;
  pl->w0 = 1.0 - w1;
  pl->r1 = w1 == 0.0 ? -1 : i0 + 1;
  pl->w1 = w1;
  const int lo = p.npml, hi = p.npml + p.nz - 1;
  return i0 >= lo && i0 <= hi && (pl->r1 < 0 || pl->r1 <= hi);
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
  if (!plane_rows(*p, p->z_src, &t) || !plane_rows(*p, p->z_rec, &t))
    return fail3(SSX_ERR_ARG, "plane depth outside the physical grid");
  const long long NZ = p->nz + 2LL * p->npml, NY = p->ny + 2LL * p->npml,
                  NX = p->nx + 2LL * p->npml;
  if (NZ > 65535 || NY * NX > (1LL << 31) || NZ * NY * NX > (1LL << 40))
    return fail3(SSX_ERR_ARG, "grid too large");
  return SSX_OK;
}

ssx_status check_model3(const ssx3_problem& p, const double* kappa, double rho, double* cmax) {
  if (!(std::isfinite(rho) && rho > 0.0)) return fail3(SSX_ERR_ARG, "rho must be finite and > 0");
  const long long n = (long long)p.nz * p.ny * p.nx;
  double kmax = 0.0;
  for (long long i = 0; i < n; ++i) {
    if (!(std::isfinite(kappa[i]) && kappa[i] > 0.0))
      return fail3(SSX_ERR_ARG, "kappa must be finite and > 0");
    kmax = std::max(kmax, kappa[i]);
  }
  *cmax = std::sqrt(kmax / rho);
  // leapfrog stability on the 3D staggered grid
  if (*cmax * p.dt / p.h > 1.0 / (std::sqrt(3.0) * weight_sum(p.order)))
    return fail3(SSX_ERR_CFL, "dt above the 3D stability bound");
  return SSX_OK;
}

Dims3 dims_of(const ssx3_problem& p) {
  return {p.nz + 2 * p.npml, p.ny + 2 * p.npml, p.nx + 2 * p.npml, p.npml};
}

size_t bytes_of(const ssx3_problem& p) {
  const Dims3 d = dims_of(p);
  const size_t n = (size_t)d.NZ * d.NY * d.NX;
  const size_t esz = p.field_dtype == SSX_F64 ? 8 : 4;
  return (8 * n + 4 * (size_t)(d.NZ + d.NY + d.NX)) * esz;
}

template <typename T>
void fill_coefs(const ssx3_problem& p, const Dims3& d, const double* kappa, double cmax,
                std::vector<T>& ck, std::vector<T>& fac) {
  const int L = p.npml;
  ck.resize((size_t)d.NZ * d.NY * d.NX);
  // the model extended into the layer by the nearest physical value
  for (int z = 0; z < d.NZ; ++z) {
    const int iz = std::min(std::max(z - L, 0), p.nz - 1);
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
  const int Ns[3] = {d.NZ, d.NY, d.NX}, ns[3] = {p.nz, p.ny, p.nx};
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

const char* at(const void* base, long long elems, size_t esz) {
  return static_cast<const char*>(base) + elems * (long long)esz;
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
  ssx_status s = check3(prob);
  if (s != SSX_OK) return s;
  if (!kappa_host) return fail3(SSX_ERR_ARG, "kappa_host is required");
  double cmax;
  s = check_model3(*prob, kappa_host, rho, &cmax);
  if (s != SSX_OK) return s;
  ssx3_ctx* c = new ssx3_ctx();
  c->prob = *prob;
  const ssx3_problem& p = c->prob;
  c->d = dims_of(p);
  c->f64 = p.field_dtype == SSX_F64;
  c->esz = c->f64 ? 8 : 4;
  c->stream = static_cast<hipStream_t>(stream);
  c->cb = p.dt / (rho * p.h);
  plane_rows(p, p.z_src, &c->src);
  plane_rows(p, p.z_rec, &c->rec);
  c->src.x0 = p.npml + (int)std::llround(p.x_src0 / p.h);
  c->src.nx = p.nsx;
  c->src.y0 = p.npml + (int)std::llround(p.y_src0 / p.h);
  c->src.ny = p.nsy;
  c->rec.x0 = p.npml + (int)std::llround(p.x_rec0 / p.h);
  c->rec.nx = p.nrx;
  c->rec.y0 = p.npml + (int)std::llround(p.y_rec0 / p.h);
  c->rec.ny = p.nry;
  const long long n = (long long)c->d.NZ * c->d.NY * c->d.NX;
  if (hipMalloc(&c->buf, bytes_of(p)) != hipSuccess) {
    delete c;
    (void)hipGetLastError();
    return fail3(SSX_ERR_OOM, "device allocation failed");
  }
  c->fields = c->buf;
  c->ck = static_cast<char*>(c->buf) + 7 * n * (long long)c->esz;
  c->fac = static_cast<char*>(c->buf) + 8 * n * (long long)c->esz;
  hipError_t e1, e2;
  if (c->f64) {
    std::vector<double> ck, fac;
    fill_coefs<double>(p, c->d, kappa_host, cmax, ck, fac);
    e1 = hipMemcpy(c->ck, ck.data(), ck.size() * 8, hipMemcpyHostToDevice);
    e2 = hipMemcpy(c->fac, fac.data(), fac.size() * 8, hipMemcpyHostToDevice);
  } else {
    std::vector<float> ck, fac;
    fill_coefs<float>(p, c->d, kappa_host, cmax, ck, fac);
    e1 = hipMemcpy(c->ck, ck.data(), ck.size() * 4, hipMemcpyHostToDevice);
    e2 = hipMemcpy(c->fac, fac.data(), fac.size() * 4, hipMemcpyHostToDevice);
  }
  if (e1 != hipSuccess || e2 != hipSuccess) {
    (void)hipFree(c->buf);
    delete c;
    return fail3(SSX_ERR_HIP, std::string("coefficient upload: ") +
                                  hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  }
  *out = c;
  return SSX_OK;
}

ssx_status ssx3_fwd(ssx3_ctx* c, const void* h, void* d) {
  if (!c || !h || !d) return fail3(SSX_ERR_ARG, "null argument");
  const ssx3_problem& p = c->prob;
  const long long n = (long long)c->d.NZ * c->d.NY * c->d.NX;
  const long long ns = (long long)p.nsx * p.nsy, nr = (long long)p.nrx * p.nry;
  S3_HIP(hipMemsetAsync(c->fields, 0, 7 * n * c->esz, c->stream));
  for (int t = 0; t < p.nt; ++t) {
    S3_HIP(ssx3::launch3_step(c->f64, p.order, false, c->fields, c->d, c->fac, c->ck, c->cb,
                              c->src, at(h, t * ns, c->esz), c->stream));
    S3_HIP(ssx3::launch3_gather(c->f64, false, c->fields, c->d, c->rec, c->fac, c->ck,
                                const_cast<char*>(at(d, t * nr, c->esz)), c->stream));
  }
  return SSX_OK;
}

ssx_status ssx3_adj(ssx3_ctx* c, const void* r, void* g) {
  if (!c || !r || !g) return fail3(SSX_ERR_ARG, "null argument");
  const ssx3_problem& p = c->prob;
  const long long n = (long long)c->d.NZ * c->d.NY * c->d.NX;
  const long long ns = (long long)p.nsx * p.nsy, nr = (long long)p.nrx * p.nry;
  S3_HIP(hipMemsetAsync(c->fields, 0, 7 * n * c->esz, c->stream));
  S3_HIP(ssx3::launch3_spread(c->f64, c->fields, c->d, c->rec, at(r, (p.nt - 1) * nr, c->esz),
                              c->stream));
  for (int t = p.nt - 1; t >= 0; --t) {
    S3_HIP(ssx3::launch3_gather(c->f64, true, c->fields, c->d, c->src, c->fac, c->ck,
                                const_cast<char*>(at(g, t * ns, c->esz)), c->stream));
    S3_HIP(ssx3::launch3_step(c->f64, p.order, true, c->fields, c->d, c->fac, c->ck, c->cb,
                              c->rec, t >= 1 ? at(r, (t - 1) * nr, c->esz) : nullptr,
                              c->stream));
  }
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
