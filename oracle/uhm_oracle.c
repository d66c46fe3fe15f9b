/*
 * CPU oracle: the paper's parallel matrix-vector products in plain C99, FP64.
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg call this file.  It shares no code with the HIP library.
 *
 *   oracle_uh_mvp_alg6  uniform H-matrix MVP, staged as Algorithm 6 (section 4.4):
 *                       a parallel loop over column clusters computes u_sigma = V_sigma^* v|_sigma;
 *                       a second parallel loop over row clusters sums the coupling products
 *                       u_tau = sum_{sigma in row(tau)} S_b u_sigma and adds U_tau u_tau, and
 *                       over dense blocks adds A|_b v|_sigma; each thread owns a copy w^(q) of
 *                       the output, and the copies are summed at the end.
 *                       The couplings are stored assembled (S_b = S_{X,b} S_{Y,b}^*), so the
 *                       product with S_b happens once, in the row loop.
 *   oracle_h_mvp_alg5   H-matrix MVP, Algorithm 5 (section 4.4): a parallel loop over
 *                       admissible blocks adds X_b (Y_b^* v|_sigma), and over dense blocks adds
 *                       A|_b v|_sigma, into per-thread copies of w that are summed at the end.
 *
 * Work is handed out dynamically from lists sorted large to small, as section 4.4
 * describes.  Vectors are in user order; the operator's cluster order is reached through
 * perm (cluster position -> user index).  Complex numbers are interleaved (re, im) pairs
 * and every stored matrix is column-major at its element offset.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef struct { double re, im; } cpx;

static inline cpx cmul(cpx a, cpx b) { cpx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cpx cmulc(cpx a, cpx b) { /* conj(a) * b */ cpx r = {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; return r; }
static inline void cacc(cpx* d, cpx a) { d->re += a.re; d->im += a.im; }

typedef struct { int64_t key; int64_t id; } item;
static int by_key_desc(const void* a, const void* b) {
  const item* x = (const item*)a; const item* y = (const item*)b;
  if (x->key != y->key) return x->key < y->key ? 1 : -1;
  return x->id < y->id ? -1 : (x->id > y->id);
}

/* y(:, r) = A x(:, r) for r < nrhs, A the uniform H-matrix.  x, y: user order, ld n. */
int oracle_uh_mvp_alg6(int64_t n, const int64_t* perm, int32_t nclusters, const int64_t* off,
                       const int64_t* size, const int32_t* rank_row, const int32_t* rank_col,
                       const int64_t* U_off, const int64_t* V_off, const double* Ud, const double* Vd,
                       int64_t nadm, const int32_t* adm_row, const int32_t* adm_col, const int64_t* S_off,
                       const double* Sd, int64_t nden, const int32_t* den_row, const int32_t* den_col,
                       const int64_t* D_off, const double* Dd, int32_t nrhs, const double* xd, double* yd,
                       int32_t nthreads) {
  const cpx* U = (const cpx*)Ud; const cpx* V = (const cpx*)Vd; const cpx* S = (const cpx*)Sd;
  const cpx* D = (const cpx*)Dd; const cpx* x = (const cpx*)xd; cpx* y = (cpx*)yd;
  if (nthreads < 1) nthreads = omp_get_max_threads();
  /* v in cluster order */
  cpx* v = (cpx*)malloc(sizeof(cpx) * n);
  /* per column cluster: u_sigma, at offset uoff[sigma] */
  int64_t* uoff = (int64_t*)malloc(sizeof(int64_t) * (nclusters + 1));
  int64_t tot = 0;
  for (int32_t c = 0; c < nclusters; ++c) { uoff[c] = tot; tot += rank_col[c]; }
  cpx* u = (cpx*)malloc(sizeof(cpx) * (tot > 0 ? tot : 1));
  /* admissible blocks grouped by row cluster */
  int64_t* rptr = (int64_t*)calloc(nclusters + 1, sizeof(int64_t));
  int64_t* rblk = (int64_t*)malloc(sizeof(int64_t) * (nadm > 0 ? nadm : 1));
  for (int64_t b = 0; b < nadm; ++b) rptr[adm_row[b] + 1]++;
  for (int32_t c = 0; c < nclusters; ++c) rptr[c + 1] += rptr[c];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (nclusters + 1));
  memcpy(fill, rptr, sizeof(int64_t) * (nclusters + 1));
  for (int64_t b = 0; b < nadm; ++b) rblk[fill[adm_row[b]]++] = b;
  /* work lists, large to small */
  item* cl = (item*)malloc(sizeof(item) * nclusters);
  int64_t ncl = 0;
  for (int32_t c = 0; c < nclusters; ++c) if (rank_col[c] > 0) { cl[ncl].key = size[c] * rank_col[c]; cl[ncl].id = c; ++ncl; }
  qsort(cl, ncl, sizeof(item), by_key_desc);
  int64_t nrow_work = 0;
  item* rw = (item*)malloc(sizeof(item) * (nclusters + nden + 1));
  for (int32_t c = 0; c < nclusters; ++c)
    if (rank_row[c] > 0 && rptr[c + 1] > rptr[c]) { rw[nrow_work].key = size[c] * rank_row[c]; rw[nrow_work].id = c; ++nrow_work; }
  for (int64_t b = 0; b < nden; ++b) { rw[nrow_work].key = size[den_row[b]] * size[den_col[b]]; rw[nrow_work].id = -1 - b; ++nrow_work; }
  qsort(rw, nrow_work, sizeof(item), by_key_desc);
  cpx* wq = (cpx*)calloc((size_t)nthreads * n, sizeof(cpx));
  int32_t lmax = 1;
  for (int32_t c = 0; c < nclusters; ++c) if (rank_row[c] > lmax) lmax = rank_row[c];

  for (int32_t r = 0; r < nrhs; ++r) {
    const cpx* xr = x + (size_t)r * n;
    for (int64_t i = 0; i < n; ++i) v[i] = xr[perm[i]];
    memset(wq, 0, sizeof(cpx) * (size_t)nthreads * n);
    /* first parallel loop: u_sigma = V_sigma^* v|_sigma */
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t t = 0; t < ncl; ++t) {
      const int32_t s = (int32_t)cl[t].id;
      const int64_t ns = size[s], ls = rank_col[s];
      const cpx* Vs = V + V_off[s];
      const cpx* vs = v + off[s];
      for (int64_t j = 0; j < ls; ++j) {
        cpx acc = {0.0, 0.0};
        for (int64_t i = 0; i < ns; ++i) cacc(&acc, cmulc(Vs[j * ns + i], vs[i]));
        u[uoff[s] + j] = acc;
      }
    }
    /* second parallel loop: row clusters and dense blocks into per-thread w^(q) */
#pragma omp parallel num_threads(nthreads)
    {
      const int q = omp_get_thread_num();
      cpx* w = wq + (size_t)q * n;
      cpx* ut = (cpx*)malloc(sizeof(cpx) * lmax);
#pragma omp for schedule(dynamic, 1)
      for (int64_t t = 0; t < nrow_work; ++t) {
        const int64_t id = rw[t].id;
        if (id >= 0) {
          const int32_t c = (int32_t)id;
          const int64_t lt = rank_row[c], nt = size[c];
          for (int64_t a = 0; a < lt; ++a) { ut[a].re = 0.0; ut[a].im = 0.0; }
          for (int64_t e = rptr[c]; e < rptr[c + 1]; ++e) {
            const int64_t b = rblk[e];
            const int32_t s = adm_col[b];
            const int64_t ls = rank_col[s];
            const cpx* Sb = S + S_off[b];
            const cpx* us = u + uoff[s];
            for (int64_t j = 0; j < ls; ++j)
              for (int64_t a = 0; a < lt; ++a) cacc(&ut[a], cmul(Sb[j * lt + a], us[j]));
          }
          const cpx* Ut = U + U_off[c];
          cpx* wt = w + off[c];
          for (int64_t a = 0; a < lt; ++a)
            for (int64_t i = 0; i < nt; ++i) cacc(&wt[i], cmul(Ut[a * nt + i], ut[a]));
        } else {
          const int64_t b = -1 - id;
          const int64_t m = size[den_row[b]], k = size[den_col[b]];
          const cpx* Db = D + D_off[b];
          const cpx* vs = v + off[den_col[b]];
          cpx* wt = w + off[den_row[b]];
          for (int64_t j = 0; j < k; ++j)
            for (int64_t i = 0; i < m; ++i) cacc(&wt[i], cmul(Db[j * m + i], vs[j]));
        }
      }
      free(ut);
    }
    /* reduction w = sum_q w^(q), scattered to user order */
    cpx* yr = y + (size_t)r * n;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
      cpx acc = {0.0, 0.0};
      for (int q = 0; q < nthreads; ++q) cacc(&acc, wq[(size_t)q * n + i]);
      yr[perm[i]] = acc;
    }
  }
  free(v); free(uoff); free(u); free(rptr); free(rblk); free(fill); free(cl); free(rw); free(wq);
  return 0;
}

/* y(:, r) = A x(:, r), A the H-matrix with A|_b = X_b Y_b^* on admissible blocks. */
int oracle_h_mvp_alg5(int64_t n, const int64_t* perm, const int64_t* off, const int64_t* size,
                      int64_t nadm, const int32_t* adm_row, const int32_t* adm_col, const int32_t* adm_rank,
                      const int64_t* X_off, const int64_t* Y_off, const double* Xd, const double* Yd,
                      int64_t nden, const int32_t* den_row, const int32_t* den_col, const int64_t* D_off,
                      const double* Dd, int32_t nrhs, const double* xd, double* yd, int32_t nthreads) {
  const cpx* X = (const cpx*)Xd; const cpx* Y = (const cpx*)Yd; const cpx* D = (const cpx*)Dd;
  const cpx* x = (const cpx*)xd; cpx* y = (cpx*)yd;
  if (nthreads < 1) nthreads = omp_get_max_threads();
  cpx* v = (cpx*)malloc(sizeof(cpx) * n);
  item* wl = (item*)malloc(sizeof(item) * (nadm + nden + 1));
  int64_t nw = 0;
  int32_t kmax = 1;
  for (int64_t b = 0; b < nadm; ++b) {
    wl[nw].key = (size[adm_row[b]] + size[adm_col[b]]) * adm_rank[b]; wl[nw].id = b; ++nw;
    if (adm_rank[b] > kmax) kmax = adm_rank[b];
  }
  for (int64_t b = 0; b < nden; ++b) { wl[nw].key = size[den_row[b]] * size[den_col[b]]; wl[nw].id = -1 - b; ++nw; }
  qsort(wl, nw, sizeof(item), by_key_desc);
  cpx* wq = (cpx*)calloc((size_t)nthreads * n, sizeof(cpx));
  for (int32_t r = 0; r < nrhs; ++r) {
    const cpx* xr = x + (size_t)r * n;
    for (int64_t i = 0; i < n; ++i) v[i] = xr[perm[i]];
    memset(wq, 0, sizeof(cpx) * (size_t)nthreads * n);
#pragma omp parallel num_threads(nthreads)
    {
      cpx* w = wq + (size_t)omp_get_thread_num() * n;
      cpx* tb = (cpx*)malloc(sizeof(cpx) * kmax);
#pragma omp for schedule(dynamic, 1)
      for (int64_t t = 0; t < nw; ++t) {
        const int64_t id = wl[t].id;
        if (id >= 0) {
          const int64_t b = id, k = adm_rank[b];
          const int64_t m = size[adm_row[b]], ns = size[adm_col[b]];
          const cpx* Xb = X + X_off[b];
          const cpx* Yb = Y + Y_off[b];
          const cpx* vs = v + off[adm_col[b]];
          cpx* wt = w + off[adm_row[b]];
          for (int64_t l = 0; l < k; ++l) {
            cpx acc = {0.0, 0.0};
            for (int64_t j = 0; j < ns; ++j) cacc(&acc, cmulc(Yb[l * ns + j], vs[j]));
            tb[l] = acc;
          }
          for (int64_t l = 0; l < k; ++l)
            for (int64_t i = 0; i < m; ++i) cacc(&wt[i], cmul(Xb[l * m + i], tb[l]));
        } else {
          const int64_t b = -1 - id;
          const int64_t m = size[den_row[b]], k = size[den_col[b]];
          const cpx* Db = D + D_off[b];
          const cpx* vs = v + off[den_col[b]];
          cpx* wt = w + off[den_row[b]];
          for (int64_t j = 0; j < k; ++j)
            for (int64_t i = 0; i < m; ++i) cacc(&wt[i], cmul(Db[j * m + i], vs[j]));
        }
      }
      free(tb);
    }
    cpx* yr = y + (size_t)r * n;
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int64_t i = 0; i < n; ++i) {
      cpx acc = {0.0, 0.0};
      for (int q = 0; q < nthreads; ++q) cacc(&acc, wq[(size_t)q * n + i]);
      yr[perm[i]] = acc;
    }
  }
  free(v); free(wl); free(wq);
  return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
