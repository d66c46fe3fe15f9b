// Host-side operator construction: kernel evaluation and adaptive cross approximation.
//
// The Helmholtz single-layer kernel g(x,y) = exp(i kappa |x-y|) / (4 pi |x-y|) (section
// 6.1) is evaluated on point pairs given in cluster order.  Admissible blocks are
// approximated by ACA with partial pivoting (the variant of Bebendorf that section 2.3
// names): rows and columns of the residual are sampled one pivot at a time, and the
// iteration stops once the newest rank-one term is small relative to the Frobenius norm
// of the running approximation.  The algebraic recompression that follows ACA (section
// 2.3) is done by the Python builder with LAPACK.
//
// Everything here runs on the host with OpenMP; nothing is on the MVP path.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include <omp.h>

namespace {

using cplx = std::complex<double>;
constexpr double kFourPi = 12.566370614359172953850573533118;

struct Geometry {
  const double* pts;  // (n, 3) row-major, cluster order
  double kappa;
  double diag;  // value used where two positions coincide (the diagonal of the matrix)
};

inline cplx kernel_at(const Geometry& g, int64_t i, int64_t j) {
  const double* a = g.pts + 3 * i;
  const double* b = g.pts + 3 * j;
  const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
  if (i == j || r == 0.0) return cplx(g.diag, 0.0);
  const double s = 1.0 / (kFourPi * r);
  return cplx(std::cos(g.kappa * r) * s, std::sin(g.kappa * r) * s);
}

struct AcaResult {
  int64_t m = 0, n = 0;
  int32_t k = 0;
  std::vector<cplx> u;  // m x k column-major: A ~ sum_l u_l v_l^T
  std::vector<cplx> v;  // n x k column-major
};

// ACA with partial pivoting on the block rows [r0, r0+m) x cols [c0, c0+n).
void aca_block(const Geometry& g, int64_t r0, int64_t m, int64_t c0, int64_t n, double eps,
               int32_t kcap, AcaResult& out) {
  out.m = m;
  out.n = n;
  out.k = 0;
  out.u.clear();
  out.v.clear();
  const int32_t kmax = static_cast<int32_t>(std::min<int64_t>({m, n, (int64_t)kcap}));
  std::vector<char> used(m, 0);
  std::vector<cplx> row(n), col(m);
  double norm2 = 0.0;  // squared Frobenius norm of the running approximation
  int64_t i = 0;
  int64_t unused = m;
  while (out.k < kmax && unused > 0) {
    const int32_t k = out.k;
    // residual row i
    for (int64_t j = 0; j < n; ++j) row[j] = kernel_at(g, r0 + i, c0 + j);
    for (int32_t l = 0; l < k; ++l) {
      const cplx ui = out.u[(size_t)l * m + i];
      const cplx* vl = out.v.data() + (size_t)l * n;
      for (int64_t j = 0; j < n; ++j) row[j] -= ui * vl[j];
    }
    used[i] = 1;
    --unused;
    int64_t jp = 0;
    double best = -1.0;
    for (int64_t j = 0; j < n; ++j) {
      const double a = std::abs(row[j]);
      if (a > best) { best = a; jp = j; }
    }
    if (!(best > 0.0)) {
      // the residual row vanishes: move on to the next unused row
      int64_t nx = -1;
      for (int64_t t = 0; t < m; ++t) if (!used[t]) { nx = t; break; }
      if (nx < 0) break;
      i = nx;
      continue;
    }
    const cplx piv = row[jp];
    // residual column jp
    for (int64_t t = 0; t < m; ++t) col[t] = kernel_at(g, r0 + t, c0 + jp);
    for (int32_t l = 0; l < k; ++l) {
      const cplx vj = out.v[(size_t)l * n + jp];
      const cplx* ul = out.u.data() + (size_t)l * m;
      for (int64_t t = 0; t < m; ++t) col[t] -= vj * ul[t];
    }
    // new term u_k v_k^T with v_k = row / pivot, u_k = col
    out.u.resize((size_t)(k + 1) * m);
    out.v.resize((size_t)(k + 1) * n);
    cplx* uk = out.u.data() + (size_t)k * m;
    cplx* vk = out.v.data() + (size_t)k * n;
    const cplx inv = 1.0 / piv;
    double nu = 0.0, nv = 0.0;
    for (int64_t t = 0; t < m; ++t) { uk[t] = col[t]; nu += std::norm(uk[t]); }
    for (int64_t j = 0; j < n; ++j) { vk[j] = row[j] * inv; nv += std::norm(vk[j]); }
    // |S_k|^2 = |S_{k-1}|^2 + 2 Re sum_l (u_l^H u_k)(v_l^H v_k) + |u_k|^2 |v_k|^2
    double cross = 0.0;
    for (int32_t l = 0; l < k; ++l) {
      const cplx* ul = out.u.data() + (size_t)l * m;
      const cplx* vl = out.v.data() + (size_t)l * n;
      cplx a(0.0, 0.0), b(0.0, 0.0);
      for (int64_t t = 0; t < m; ++t) a += std::conj(ul[t]) * uk[t];
      for (int64_t j = 0; j < n; ++j) b += std::conj(vl[j]) * vk[j];
      cross += (a * b).real();
    }
    norm2 += 2.0 * cross + nu * nv;
    out.k = k + 1;
    if (std::sqrt(nu * nv) <= eps * std::sqrt(std::max(norm2, 0.0))) break;
    // next pivot row: largest entry of u_k among unused rows
    int64_t nx = -1;
    double bu = -1.0;
    for (int64_t t = 0; t < m; ++t) {
      if (used[t]) continue;
      const double a = std::abs(uk[t]);
      if (a > bu) { bu = a; nx = t; }
    }
    if (nx < 0) break;
    i = nx;
  }
}

struct AcaBatch {
  std::vector<AcaResult> res;
};

}  // namespace

extern "C" {

// Dense blocks: block b covers rows [roff[b], roff[b]+rsize[b]) and columns
// [coff[b], coff[b]+csize[b]) of the cluster-ordered matrix and is written column-major
// at out + 2*dst[b] (interleaved complex128).
int uhmb_dense_blocks(const double* pts, double kappa, double diag, int64_t nb, const int64_t* roff,
                      const int64_t* rsize, const int64_t* coff, const int64_t* csize,
                      const int64_t* dst, double* out) {
  const Geometry g{pts, kappa, diag};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t b = 0; b < nb; ++b) {
    cplx* o = reinterpret_cast<cplx*>(out) + dst[b];
    const int64_t m = rsize[b], n = csize[b];
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < m; ++i) o[j * m + i] = kernel_at(g, roff[b] + i, coff[b] + j);
  }
  return 0;
}

// Run ACA on nb blocks in parallel (largest first).  Returns an opaque handle that owns
// the factors until uhmb_aca_free; ranks go to k_out[nb].
void* uhmb_aca_run(const double* pts, double kappa, double diag, int64_t nb, const int64_t* roff,
                   const int64_t* rsize, const int64_t* coff, const int64_t* csize, double eps,
                   int32_t kcap, int32_t* k_out) {
  AcaBatch* h = new (std::nothrow) AcaBatch;
  if (!h) return nullptr;
  h->res.resize(nb);
  std::vector<int64_t> order(nb);
  for (int64_t b = 0; b < nb; ++b) order[b] = b;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    return rsize[a] + csize[a] > rsize[b] + csize[b];
  });
  const Geometry g{pts, kappa, diag};
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nb; ++t) {
    const int64_t b = order[t];
    aca_block(g, roff[b], rsize[b], coff[b], csize[b], eps, kcap, h->res[b]);
  }
  for (int64_t b = 0; b < nb; ++b) k_out[b] = h->res[b].k;
  return h;
}

// Copy the factors of blocks idx[0..cnt) into zero-padded batches:
// X[c] (m x kp, row-major) = u, Y[c] (n x kp, row-major) = conj(v), so A|_b ~ X Y^H.
int uhmb_aca_copy(void* handle, int64_t cnt, const int64_t* idx, int64_t m, int64_t n, int64_t kp,
                  double* X, double* Y) {
  AcaBatch* h = static_cast<AcaBatch*>(handle);
  cplx* Xc = reinterpret_cast<cplx*>(X);
  cplx* Yc = reinterpret_cast<cplx*>(Y);
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t c = 0; c < cnt; ++c) {
    const AcaResult& r = h->res[idx[c]];
    cplx* xo = Xc + (size_t)c * m * kp;
    cplx* yo = Yc + (size_t)c * n * kp;
    std::memset(static_cast<void*>(xo), 0, sizeof(cplx) * m * kp);
    std::memset(static_cast<void*>(yo), 0, sizeof(cplx) * n * kp);
    if (r.m > m || r.n > n || r.k > kp) continue;
    for (int32_t l = 0; l < r.k; ++l) {
      for (int64_t i = 0; i < r.m; ++i) xo[i * kp + l] = r.u[(size_t)l * r.m + i];
      for (int64_t j = 0; j < r.n; ++j) yo[j * kp + l] = std::conj(r.v[(size_t)l * r.n + j]);
    }
  }
  return 0;
}

void uhmb_aca_free(void* handle) { delete static_cast<AcaBatch*>(handle); }

// ACA of one block on the calling thread (no OpenMP), for construction schedules that
// approximate blocks on demand.  X (m x kcap, row-major) = u and Y (n x kcap, row-major) =
// conj(v), so A|_b ~ X Y^H in the first k columns (the rest zero); returns k, or -1 when
// kcap < 1.
int32_t uhmb_aca_block(const double* pts, double kappa, double diag, int64_t r0, int64_t m, int64_t c0,
                       int64_t n, double eps, int32_t kcap, double* X, double* Y) {
  if (kcap < 1) return -1;
  const Geometry g{pts, kappa, diag};
  AcaResult r;
  aca_block(g, r0, m, c0, n, eps, kcap, r);
  cplx* xo = reinterpret_cast<cplx*>(X);
  cplx* yo = reinterpret_cast<cplx*>(Y);
  std::memset(static_cast<void*>(xo), 0, sizeof(cplx) * m * kcap);
  std::memset(static_cast<void*>(yo), 0, sizeof(cplx) * n * kcap);
  for (int32_t l = 0; l < r.k; ++l) {
    for (int64_t i = 0; i < m; ++i) xo[i * kcap + l] = r.u[(size_t)l * m + i];
    for (int64_t j = 0; j < n; ++j) yo[j * kcap + l] = std::conj(r.v[(size_t)l * n + j]);
  }
  return r.k;
}

// Scaled copies of complex128 matrices, for laying out the agglomerated block rows X_tau
// and the H-matrix factors: for each record e and i < rows, q < cols,
//   dst[i * drs + q * dcs] = f(src[i * srs + q * scs]) * scale[q],
// f = conj when conj != 0, no scaling when scale is 0, zeros written when src is 0.
// Addresses are byte addresses, strides count complex elements.  The records are spread
// over the OpenMP threads; their destinations must not overlap.
struct uhmb_copy {
  uint64_t src, dst, scale;
  int64_t srs, scs, drs, dcs;
  int32_t rows, cols, conj, pad;
};

int uhmb_scaled_copy(const uhmb_copy* rec, int64_t nrec) {
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t e = 0; e < nrec; ++e) {
    const uhmb_copy r = rec[e];
    cplx* d = reinterpret_cast<cplx*>(r.dst);
    const cplx* sp = reinterpret_cast<const cplx*>(r.src);
    const double* sc = reinterpret_cast<const double*>(r.scale);
    auto value = [&](int64_t i, int64_t q) {
      if (!sp) return cplx(0.0, 0.0);
      cplx v = sp[i * r.srs + q * r.scs];
      if (r.conj) v = std::conj(v);
      return sc ? cplx(v.real() * sc[q], v.imag() * sc[q]) : v;
    };
    if (r.dcs == 1) {  // rows of the destination contiguous
      for (int64_t i = 0; i < r.rows; ++i)
        for (int64_t q = 0; q < r.cols; ++q) d[i * r.drs + q] = value(i, q);
    } else {
      for (int64_t q = 0; q < r.cols; ++q)
        for (int64_t i = 0; i < r.rows; ++i) d[i * r.drs + q * r.dcs] = value(i, q);
    }
  }
  return 0;
}

int uhmb_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
