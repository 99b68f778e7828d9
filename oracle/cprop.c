/*
 * cprop.c -- the oracle's time stepping written as plain C loops (FP64).
 *
 * TEST INFRASTRUCTURE ONLY: this engine belongs to the oracle package and is
 * loaded only by its Python wrapper (oracle/cengine.py), which the tests, the
 * golden-data scripts and the benchmark's CPU-baseline leg may use.  The
 * product library never links or calls it, and it shares no code with it.
 *
 * It computes exactly what oracle/prop.py computes -- the same sub-updates
 * in the same order, each stencil sum accumulated term by term in the order
 * of the NumPy version (the file is built with -ffp-contract=off), so the
 * two agree to rounding -- but as loops over the cells of each sub-update,
 * with the rows of a sub-update shared out over OpenMP threads (every cell
 * of a sub-update is independent of the others, so the result does not
 * depend on the thread count).
 *
 * Scheme (W. W. Symes, "Efficient Computation of Extended Surface Sources",
 * Numerical Examples: staggered grid, order 2 in time and 2k in space,
 * absorbing layer on all sides, linear interpolation for sampling and its
 * transpose for injection).  Step n -> n+1, with p = p_x + p_z:
 *
 *   v_x <- a_x,h v_x - (b_x,h Cb) D_x^+ p
 *   v_z <- a_z,h v_z - (b_z,h Cb) (D_z^+ p - E_f f[n])
 *   p_x <- a_x,n p_x - (b_x,n Ck) D_x^- v_x
 *   p_z <- a_z,n p_z - (b_z,n Ck) (D_z^- v_z - E_h h[n])
 *   P[n] = R_p (p_x + p_z),  V[n] = R_vz v_z
 *
 * D^+ and D^- omit 1/h (folded into Cb = dt/(rho h) and Ck = dt kappa/h);
 * fields outside the array are zero.  The transpose runs the transposed
 * sub-updates in reverse order (Operators section, adjoint-state identity;
 * Appendix A).
 */
#include <stdlib.h>
#include <string.h>

/* A sampled line: one or two rows with interpolation weights, n columns. */
typedef struct {
  int nrows;
  int row[2];
  double w[2];
  int n;
  const int* cols;
} oc_line;

/* Layer factors of one grid: x arrays of length NX, z arrays of length NZ. */
typedef struct {
  const double *axn, *bxn, *axh, *bxh;
  const double *azn, *bzn, *azh, *bzh;
} oc_pml;

#define AT(a, i, j) (a)[(size_t)(i) * (size_t)NX + (size_t)(j)]

/* out[j] = sum_m c_m (u[j + op_m] - u[j + on_m]) along x (axis 1) or z
 * (axis 0), zero outside the array: the terms are added one at a time,
 * + c_m u[j + op_m] then + (-c_m) u[j + on_m], for m = 1..k.  Terms that
 * fall outside the array are skipped; where none does (the bulk of each
 * row or of the rows) the same sum is written without the tests. */
static inline double term_sum(int k, const double* c, const int* op, const int* on,
                              const double* u, long stride) {
  double s = 0.0;
  for (int m = 0; m < k; ++m) {
    s += c[m] * u[op[m] * stride];
    s += (-c[m]) * u[on[m] * stride];
  }
  return s;
}

static void shift_sum(int NZ, int NX, int k, const double* c, const int* op, const int* on,
                      int axis, const double* u, double* out) {
  int lo = 0, hi = 0;  /* offsets span [lo, hi] */
  for (int m = 0; m < k; ++m) {
    if (op[m] < lo) lo = op[m];
    if (on[m] < lo) lo = on[m];
    if (op[m] > hi) hi = op[m];
    if (on[m] > hi) hi = on[m];
  }
#pragma omp parallel for schedule(static)
  for (int i = 0; i < NZ; ++i) {
    const int row_inner = axis == 1 || (i + lo >= 0 && i + hi < NZ);
    const int j0 = axis == 1 ? -lo : 0, j1 = axis == 1 ? NX - hi : NX;
    for (int j = 0; j < NX; ++j) {
      if (row_inner && j >= j0 && j < j1) {
        /* no term leaves the array for j in [j0, j1) */
        const long stride = axis == 1 ? 1 : NX;
        const double* base = &AT(u, i, 0);
        if (k == 2) {
          for (; j < j1; ++j) AT(out, i, j) = term_sum(2, c, op, on, base + j, stride);
        } else if (k == 4) {
          for (; j < j1; ++j) AT(out, i, j) = term_sum(4, c, op, on, base + j, stride);
        } else {
          for (; j < j1; ++j) AT(out, i, j) = term_sum(k, c, op, on, base + j, stride);
        }
        --j;
        continue;
      }
      double s = 0.0;
      for (int m = 0; m < k; ++m) {
        const int offs[2] = {op[m], on[m]};
        const double cm[2] = {c[m], -c[m]};
        for (int t = 0; t < 2; ++t) {
          const int ii = axis == 0 ? i + offs[t] : i;
          const int jj = axis == 1 ? j + offs[t] : j;
          if (ii < 0 || ii >= NZ || jj < 0 || jj >= NX) continue;
          s += cm[t] * AT(u, ii, jj);
        }
      }
      AT(out, i, j) = s;
    }
  }
}

/* D^+: op = m, on = 1 - m;  D^-: op = m - 1, on = -m.  Their transposes
 * negate both offsets (out_T[i] += c u[i - o] for each term out[j] += c
 * u[j + o]). */
static void dplus(int NZ, int NX, int k, const double* c, int axis, const double* u,
                  double* out) {
  int op[8], on[8];
  for (int m = 1; m <= k; ++m) { op[m - 1] = m; on[m - 1] = 1 - m; }
  shift_sum(NZ, NX, k, c, op, on, axis, u, out);
}
static void dminus(int NZ, int NX, int k, const double* c, int axis, const double* u,
                   double* out) {
  int op[8], on[8];
  for (int m = 1; m <= k; ++m) { op[m - 1] = m - 1; on[m - 1] = -m; }
  shift_sum(NZ, NX, k, c, op, on, axis, u, out);
}
static void dplus_T(int NZ, int NX, int k, const double* c, int axis, const double* u,
                    double* out) {
  int op[8], on[8];
  for (int m = 1; m <= k; ++m) { op[m - 1] = -m; on[m - 1] = m - 1; }
  shift_sum(NZ, NX, k, c, op, on, axis, u, out);
}
static void dminus_T(int NZ, int NX, int k, const double* c, int axis, const double* u,
                     double* out) {
  int op[8], on[8];
  for (int m = 1; m <= k; ++m) { op[m - 1] = 1 - m; on[m - 1] = m; }
  shift_sum(NZ, NX, k, c, op, on, axis, u, out);
}

/* out[r, cols] += (scale w_r) values, for each row of the line */
static void spread_add(int NX, const oc_line* l, const double* values, double* out,
                       double scale) {
  for (int t = 0; t < l->nrows; ++t) {
    const double sw = scale * l->w[t];
    for (int q = 0; q < l->n; ++q) AT(out, l->row[t], l->cols[q]) += sw * values[q];
  }
}

/* out = sum_r w_r field[r, cols] (linear interpolation) */
static void gather(int NX, const oc_line* l, const double* field, double* out) {
  for (int q = 0; q < l->n; ++q) out[q] = 0.0;
  for (int t = 0; t < l->nrows; ++t)
    for (int q = 0; q < l->n; ++q) out[q] += l->w[t] * AT(field, l->row[t], l->cols[q]);
}

/* gather of the product (fac[i] Cmul[i][j]) field[i][j], the products formed
 * per cell as in the vector form (bz (Ck) p), Cmul a scalar when cs != 0 */
static void gather_scaled(int NX, const oc_line* l, const double* fac_z, const double* Cmul,
                          double cs, const double* field, double* out) {
  for (int q = 0; q < l->n; ++q) out[q] = 0.0;
  for (int t = 0; t < l->nrows; ++t) {
    const int i = l->row[t];
    for (int q = 0; q < l->n; ++q) {
      const int j = l->cols[q];
      const double f = Cmul ? fac_z[i] * AT(Cmul, i, j) : fac_z[i] * cs;
      out[q] += l->w[t] * (f * AT(field, i, j));
    }
  }
}

static double* zalloc(size_t n) { return (double*)calloc(n, sizeof(double)); }

/* Forward run of nt steps from rest (see the file header).  h / f: injected
 * traces [nt][line n] (NULL: none); P / V: recorded traces (NULL: none).
 * Returns 0, or -1 when memory runs out. */
int oc_forward(int NZ, int NX, int k, const double* c, double Cb, const double* Ck,
               const oc_pml* pm, int nt, const oc_line* hl, const double* h,
               const oc_line* fl, const double* f, const oc_line* rp, double* P,
               const oc_line* rv, double* V) {
  const size_t N = (size_t)NZ * (size_t)NX;
  double *vx = zalloc(N), *vz = zalloc(N), *px = zalloc(N), *pz = zalloc(N);
  double *p = zalloc(N), *d = zalloc(N);
  int ok = vx && vz && px && pz && p && d;
  for (int n = 0; ok && n < nt; ++n) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) AT(p, i, j) = AT(px, i, j) + AT(pz, i, j);
    /* v_x */
    dplus(NZ, NX, k, c, 1, p, d);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j)
        AT(vx, i, j) = pm->axh[j] * AT(vx, i, j) - (pm->bxh[j] * Cb) * AT(d, i, j);
    /* v_z */
    dplus(NZ, NX, k, c, 0, p, d);
    if (fl) spread_add(NX, fl, f + (size_t)n * fl->n, d, -1.0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j)
        AT(vz, i, j) = pm->azh[i] * AT(vz, i, j) - (pm->bzh[i] * Cb) * AT(d, i, j);
    /* p_x */
    dminus(NZ, NX, k, c, 1, vx, d);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j)
        AT(px, i, j) = pm->axn[j] * AT(px, i, j) - (pm->bxn[j] * AT(Ck, i, j)) * AT(d, i, j);
    /* p_z */
    dminus(NZ, NX, k, c, 0, vz, d);
    if (hl) spread_add(NX, hl, h + (size_t)n * hl->n, d, -1.0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j)
        AT(pz, i, j) = pm->azn[i] * AT(pz, i, j) - (pm->bzn[i] * AT(Ck, i, j)) * AT(d, i, j);
    if (rp) {
#pragma omp parallel for schedule(static)
      for (int i = 0; i < NZ; ++i)
        for (int j = 0; j < NX; ++j) AT(p, i, j) = AT(px, i, j) + AT(pz, i, j);
      gather(NX, rp, p, P + (size_t)n * rp->n);
    }
    if (rv) gather(NX, rv, vz, V + (size_t)n * rv->n);
  }
  free(vx); free(vz); free(px); free(pz); free(p); free(d);
  return ok ? 0 : -1;
}

/* Exact transpose of oc_forward as a map from (h, f) to (P, V): a and b are
 * the adjoint inputs in the P and V slots ([nt][line n], NULL: none); hb and
 * fb receive the adjoint outputs of the h and f slots (NULL: not wanted). */
int oc_adjoint(int NZ, int NX, int k, const double* c, double Cb, const double* Ck,
               const oc_pml* pm, int nt, const oc_line* hl, double* hb, const oc_line* fl,
               double* fb, const oc_line* rp, const double* a, const oc_line* rv,
               const double* b) {
  const size_t N = (size_t)NZ * (size_t)NX;
  double *vxb = zalloc(N), *vzb = zalloc(N), *pxb = zalloc(N), *pzb = zalloc(N);
  double *tmp = zalloc(N), *d = zalloc(N), *t = zalloc(N);
  int ok = vxb && vzb && pxb && pzb && tmp && d && t;
  for (int n = nt - 1; ok && n >= 0; --n) {
    /* recording P[n] = R_p (p_x + p_z), V[n] = R_vz v_z */
    if (rp) {
      spread_add(NX, rp, a + (size_t)n * rp->n, pxb, 1.0);
      spread_add(NX, rp, a + (size_t)n * rp->n, pzb, 1.0);
    }
    if (rv) spread_add(NX, rv, b + (size_t)n * rv->n, vzb, 1.0);
    /* p_z update: its source slot, then the transposed D^- terms */
    if (hl && hb) gather_scaled(NX, hl, pm->bzn, Ck, 0.0, pzb, hb + (size_t)n * hl->n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) AT(tmp, i, j) = (pm->bxn[j] * AT(Ck, i, j)) * AT(pxb, i, j);
    dminus_T(NZ, NX, k, c, 1, tmp, d);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) AT(vxb, i, j) = AT(vxb, i, j) - AT(d, i, j);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) AT(tmp, i, j) = (pm->bzn[i] * AT(Ck, i, j)) * AT(pzb, i, j);
    dminus_T(NZ, NX, k, c, 0, tmp, d);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) {
        AT(vzb, i, j) = AT(vzb, i, j) - AT(d, i, j);
        AT(pxb, i, j) = pm->axn[j] * AT(pxb, i, j);
        AT(pzb, i, j) = pm->azn[i] * AT(pzb, i, j);
      }
    /* v_z update: its source slot, then the transposed D^+ terms */
    if (fl && fb) gather_scaled(NX, fl, pm->bzh, NULL, Cb, vzb, fb + (size_t)n * fl->n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) AT(tmp, i, j) = (pm->bxh[j] * Cb) * AT(vxb, i, j);
    dplus_T(NZ, NX, k, c, 1, tmp, t);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) AT(tmp, i, j) = (pm->bzh[i] * Cb) * AT(vzb, i, j);
    dplus_T(NZ, NX, k, c, 0, tmp, d);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < NZ; ++i)
      for (int j = 0; j < NX; ++j) {
        const double tt = -(AT(t, i, j) + AT(d, i, j));
        AT(pxb, i, j) = AT(pxb, i, j) + tt;
        AT(pzb, i, j) = AT(pzb, i, j) + tt;
        AT(vxb, i, j) = pm->axh[j] * AT(vxb, i, j);
        AT(vzb, i, j) = pm->azh[i] * AT(vzb, i, j);
      }
  }
  free(vxb); free(vzb); free(pxb); free(pzb); free(tmp); free(d); free(t);
  return ok ? 0 : -1;
}
