// Alg. 2's per-cluster factorisation on the GPU (section 4.2), for a batch of clusters.
//
// For a cluster tau, Alg. 2 takes the SVD of the thin factor X_tau (n_tau x k_tau: the
// scaled left factors of the blocks in tau's block row) and keeps the left singular
// vectors whose singular values exceed eps * sigma_1.  They form U_tau, and U_tau^* X_tau =
// Sigma V^* gives the rows from which the couplings follow.  The SVD is taken in four
// steps, each a batched launch over the clusters of one shape:
//
//  1. Householder QR with column pivoting, X Pi = Q [R; 0] + (trailing part), stopped once
//     the trailing part's Frobenius norm T is at most tol * ||X||_F.  Then X = Q_p B + E with
//     B = R Pi^T = Q_p^* X (p x k) and E = (I - Q_p Q_p^*) X, ||E||_F = T.  The range of E is
//     orthogonal to that of Q_p, so X^* X = B^* B + E^* E and
//       sigma_i(B)^2 <= sigma_i(X)^2 <= sigma_i(B)^2 + T^2:
//     near the rank threshold eps sigma_1 a singular value moves by at most T^2 / (2 eps
//     sigma_1).  For the same reason the projection error of the basis U taken from B is
//     at most sqrt(sigma_{l+1}(X)^2 + T^2) in the 2-norm, and its Frobenius norm is exactly
//     sqrt(sum_{i>l} sigma_i(B)^2 + T^2).  With tol^2 about 1e-16 eps the rank test on B is
//     the one a full SVD of X takes, up to rounding.  One launch per step; every workgroup of a matrix
//     recomputes the pivot (largest remaining column norm, lowest index on ties) and the
//     trailing sum in the same order, so all of them take the same decisions.  Columns are
//     never moved: a pivot column is retired (norm marker -1) and R is kept in the original
//     column order, which is B itself.
//  2. Unpivoted Householder QR of B^* = Q2 R2, R2 p x p (the same step kernel).
//  3. One-sided (Hestenes) Jacobi on the columns of R2, with the rotations accumulated in J:
//     R2 J = W Sigma, so B = R2^* Q2^* = J Sigma (Q2 W)^*: the left singular vectors of B are
//     the columns of J and its singular values are the column norms.  Round-robin pairs, one
//     wavefront per pair.  The accumulated rotations lose orthogonality at the level of
//     1e-12, so the kept columns of J are orthonormalised again (classical Gram-Schmidt
//     applied twice, largest singular value first).
//  4. U = Q_p [J_l; 0] (the reflectors of step 1 applied in reverse order, the columns held
//     in registers) and Sigma V^* = J_l^* B.  The Frobenius projection error is exact:
//     ||X - U U^* X||_F^2 = sum of the dropped sigma_i(B)^2 + T^2.
#include "uhm_internal.h"

#include <climits>
#include <cmath>

namespace uhm_detail {
namespace {

constexpr int kFacMaxP = 2048;      // largest kept QR rank (columns of J)
constexpr int kFacMaxRows = 16384;  // largest cluster: 16 rows per thread in the U kernel
constexpr int kStepThreads = 256;
constexpr int kStepCols = 16;  // columns per workgroup in a QR step: 4 per wavefront
constexpr int kBigThreads = 1024;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__device__ __forceinline__ double2 cdotc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// xor butterfly: every lane ends with the same bits
__device__ __forceinline__ double fwave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Per-matrix workspace regions (offsets in doubles from the matrix's base).
struct FacWs {
  double* base;
  int64_t per;
  int64_t o_w, o_om, o_c, o_cq, o_r2, o_j, o_nu, o_ord, o_st;
  __host__ __device__ double* mat(int c) const { return base + (int64_t)c * per; }
  __host__ __device__ double2* W(int c) const { return reinterpret_cast<double2*>(mat(c) + o_w); }
  __host__ __device__ double* om(int c) const { return mat(c) + o_om; }
  __host__ __device__ double2* C(int c) const { return reinterpret_cast<double2*>(mat(c) + o_c); }
  // a second copy of B^*, which the QR of B^* consumes
  __host__ __device__ double2* Cq(int c) const { return reinterpret_cast<double2*>(mat(c) + o_cq); }
  __host__ __device__ double2* R2(int c) const { return reinterpret_cast<double2*>(mat(c) + o_r2); }
  __host__ __device__ double2* J(int c) const { return reinterpret_cast<double2*>(mat(c) + o_j); }
  __host__ __device__ double* nu(int c) const { return mat(c) + o_nu; }
  __host__ __device__ int32_t* ord(int c) const { return reinterpret_cast<int32_t*>(mat(c) + o_ord); }
  // st: [0] p (steps of the pivoted QR), [1] its stop flag, [2] steps of the second QR,
  // [3] its stop flag, [4] Jacobi sweeps, [5] Jacobi did not converge, [6] rank l,
  // [7] the pivoted QR reached pmax before the tolerance;
  // as doubles from st + 8: [0] ||X||_F^2, [1] T^2
  __host__ __device__ int32_t* st(int c) const { return reinterpret_cast<int32_t*>(mat(c) + o_st); }
  __host__ __device__ double* fro(int c) const { return mat(c) + o_st + 8; }
};

int64_t round_up(int64_t x) { return (x + 31) / 32 * 32; }

FacWs layout(double* base, int32_t m, int32_t n, int32_t P) {
  FacWs w{};
  w.base = base;
  int64_t o = 0;
  w.o_w = o;
  o += round_up(2 * (int64_t)P * m);
  w.o_om = o;
  o += round_up(P);
  w.o_c = o;
  o += round_up(2 * (int64_t)n * P);
  w.o_cq = o;
  o += round_up(2 * (int64_t)n * P);
  w.o_r2 = o;
  o += round_up(2 * (int64_t)P * P);
  w.o_j = o;
  o += round_up(2 * (int64_t)P * P);
  w.o_nu = o;
  o += round_up(2 * (int64_t)std::max(n, P));
  w.o_ord = o;
  o += round_up((P + 1) / 2);
  w.o_st = o;
  o += 32;
  w.per = o;
  return w;
}

// Squared column norms of a rows x cols matrix (lda = rows) into nu's first buffer: one
// wavefront per column, kStepCols columns per workgroup.
__global__ __launch_bounds__(kStepThreads) void k_fac_norms(const double2* __restrict__ A, int64_t a_stride,
                                                            int32_t rows, int32_t cols, FacWs ws) {
  const int c = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double2* Am = A + (int64_t)c * a_stride;
  double* nu = ws.nu(c);
  for (int q = 0; q < kStepCols / 4; ++q) {
    const int j = blockIdx.x * kStepCols + wv * (kStepCols / 4) + q;
    if (j >= cols) break;
    const double2* y = Am + (int64_t)j * rows;
    double s = 0.0;
    for (int i = lane; i < rows; i += 64) {
      const double2 v = y[i];
      s += v.x * v.x + v.y * v.y;
    }
    s = fwave_sum(s);
    if (lane == 0) nu[j] = s;
  }
}

struct QrStep {
  double2* A;  // rows x cols per matrix, column-major (lda = rows), updated in place
  int64_t a_stride;
  int32_t rows, cols;
  int32_t which;    // 0: the pivoted QR of X (state st[0..1]); 1: the QR of B^* (st[2..3])
  int32_t kcap;     // step limit (the pivoted QR also stops at the tolerance)
  double tol2;      // pivoted: stop when T^2 <= tol2 * ||X||_F^2
  int32_t keep_w;   // store the reflectors (pivoted QR)
  // R[k][j] goes to out[k * rs + j * cs] of the matrix's R area, conjugated if rconj
  int32_t rs, cs, rconj;
};

// One Householder step k for every matrix of the batch.  Grid (ceil(cols / 16), batch).
// The reflector of step k is P = I - omega w w^*, w = x - beta e_k on rows k.., x the pivot
// column, beta = -e^{i arg x_k} ||x|| (so that w_k carries no cancellation), omega =
// 1 / (||x|| (||x|| + |x_k|)); P x = beta e_k.
__global__ __launch_bounds__(kStepThreads) void k_qr_step(QrStep a, FacWs ws, int32_t k) {
  const int c = blockIdx.y;
  int32_t* st = ws.st(c) + 2 * a.which;
  if (st[1]) return;  // stopped in an earlier step
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const double* nu = ws.nu(c) + (k & 1) * (int64_t)a.cols;
  double* nu2 = ws.nu(c) + ((k + 1) & 1) * (int64_t)a.cols;
  const int32_t lim = a.which == 0 ? a.kcap : min(a.kcap, ws.st(c)[0]);

  // trailing sum and pivot over the live columns, in one fixed order
  __shared__ double s_sum[kStepThreads], s_mx[kStepThreads];
  __shared__ int s_ix[kStepThreads];
  double sum = 0.0, mx = -1.0;
  int ix = INT_MAX;
  for (int j = tid; j < a.cols; j += kStepThreads) {
    const double v = nu[j];
    if (v >= 0.0) {
      sum += v;
      if (v > mx) {
        mx = v;
        ix = j;
      }
    }
  }
  s_sum[tid] = sum;
  s_mx[tid] = mx;
  s_ix[tid] = ix;
  __syncthreads();
  for (int s = kStepThreads / 2; s > 0; s >>= 1) {
    if (tid < s) {
      s_sum[tid] += s_sum[tid + s];
      const double m2 = s_mx[tid + s];
      const int i2 = s_ix[tid + s];
      if (m2 > s_mx[tid] || (m2 == s_mx[tid] && i2 < s_ix[tid])) {
        s_mx[tid] = m2;
        s_ix[tid] = i2;
      }
    }
    __syncthreads();
  }
  const double tr = s_sum[0];
  double* fro = ws.fro(c);
  const double f2 = k == 0 ? tr : fro[0];
  const bool piv_mode = a.which == 0;
  const bool stop = k >= lim || k >= a.rows || (piv_mode && (tr <= a.tol2 * f2 || s_mx[0] <= 0.0));
  if (stop) {
    if (blockIdx.x == 0 && tid == 0) {
      st[0] = k;
      st[1] = 1;
      if (piv_mode) {
        fro[0] = f2;
        fro[1] = tr;
        // the step cap (pmax < min(rows, cols)) came before the tolerance
        ws.st(c)[7] = (k < a.rows && k < a.cols && !(tr <= a.tol2 * f2 || s_mx[0] <= 0.0)) ? 1 : 0;
      }
    }
    return;
  }
  if (piv_mode && k == 0 && blockIdx.x == 0 && tid == 0) fro[0] = tr;
  const int piv = piv_mode ? s_ix[0] : k;

  double2* Am = a.A + (int64_t)c * a.a_stride;
  const double2* x = Am + (int64_t)piv * a.rows;
  const double nx = sqrt(fmax(nu[piv], 0.0));
  const double2 al = x[k];
  const double aa = hypot(al.x, al.y);
  const double2 ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
  const double2 beta = make_double2(-ph.x * nx, -ph.y * nx);
  const double2 wk = make_double2(ph.x * (aa + nx), ph.y * (aa + nx));
  const double om = nx > 0.0 ? 1.0 / (nx * (nx + aa)) : 0.0;
  double2* R = a.which == 0 ? ws.C(c) : ws.R2(c);
  double2* Rq = a.which == 0 ? ws.Cq(c) : nullptr;

  for (int q = 0; q < kStepCols / 4; ++q) {
    const int j = blockIdx.x * kStepCols + wv * (kStepCols / 4) + q;
    if (j >= a.cols) break;
    const int64_t ro = (int64_t)k * a.rs + (int64_t)j * a.cs;
    if (j == piv) {
      if (a.keep_w) {
        double2* w = ws.W(c) + (int64_t)k * a.rows;
        for (int i = lane; i < a.rows; i += 64) w[i] = i < k ? make_double2(0.0, 0.0) : (i == k ? wk : x[i]);
        if (lane == 0) ws.om(c)[k] = om;
      }
      if (lane == 0) {
        R[ro] = a.rconj ? cconj(beta) : beta;
        if (Rq) Rq[ro] = R[ro];
        nu2[j] = -1.0;
      }
      continue;
    }
    if (nu[j] < 0.0) {  // retired in an earlier step: R is upper triangular in pivot order
      if (lane == 0) {
        R[ro] = make_double2(0.0, 0.0);
        if (Rq) Rq[ro] = make_double2(0.0, 0.0);
        nu2[j] = -1.0;
      }
      continue;
    }
    double2* y = Am + (int64_t)j * a.rows;
    double sr = 0.0, si = 0.0;
    for (int i = k + lane; i < a.rows; i += 64) {
      const double2 wi = i == k ? wk : x[i];
      const double2 t = cdotc(wi, y[i]);
      sr += t.x;
      si += t.y;
    }
    sr = fwave_sum(sr);
    si = fwave_sum(si);
    const double2 f = make_double2(om * sr, om * si);
    double nn = 0.0;
    double2 rk = make_double2(0.0, 0.0);
    for (int i = k + lane; i < a.rows; i += 64) {
      const double2 wi = i == k ? wk : x[i];
      const double2 fw = cmul(f, wi);
      double2 v = y[i];
      v.x -= fw.x;
      v.y -= fw.y;
      y[i] = v;
      if (i == k)
        rk = v;
      else
        nn += v.x * v.x + v.y * v.y;
    }
    nn = fwave_sum(nn);
    if (lane == 0) {  // lane 0 holds row k
      R[ro] = a.rconj ? cconj(rk) : rk;
      if (Rq) Rq[ro] = R[ro];
      nu2[j] = nn;
    }
  }
}

// One-sided Jacobi on the p x p matrix R2 (ld P), one workgroup of 16 wavefronts per
// matrix.  Round r of a sweep pairs the columns by the circle method (index 0 fixed, the
// others rotated), so the pairs of a round are disjoint and one wavefront takes each.  A
// pair (i, j) with Gram entries alpha, beta, gamma is rotated when |gamma| > tol sqrt(alpha
// beta): with e = gamma / |gamma|, zeta = (beta - alpha) / (2 |gamma|) and t the smaller
// root of t^2 + 2 zeta t - 1 = 0, c = 1 / sqrt(1 + t^2), s = c t,
//   a_i <- c a_i - s conj(e) a_j,   a_j <- s e a_i + c a_j,
// which makes a_i^* a_j vanish; the same rotation is applied to J.
__global__ __launch_bounds__(kBigThreads) void k_fac_jacobi(FacWs ws, int32_t P, double tol, int32_t max_sweeps) {
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int32_t* st = ws.st(c);
  const int p = st[0];
  double2* R = ws.R2(c);
  double2* V = ws.J(c);
  for (int64_t q = tid; q < (int64_t)P * P; q += kBigThreads) {
    const int r = (int)(q % P), col = (int)(q / P);
    V[q] = make_double2(r == col && r < p ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  __shared__ int s_rot;
  const int pp = p + (p & 1);
  int sweep = 0;
  bool conv = p < 2;
  while (!conv && sweep < max_sweeps) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < pp - 1; ++r) {
      for (int q = wv; q < pp / 2; q += kBigThreads / 64) {
        const int a0 = q == 0 ? 0 : (r + q - 1) % (pp - 1) + 1;
        const int b0 = (r + (pp - 1 - q) - 1) % (pp - 1) + 1;
        const int i = min(a0, b0), j = max(a0, b0);
        if (j >= p) continue;
        double2* ci = R + (int64_t)i * P;
        double2* cj = R + (int64_t)j * P;
        double al = 0.0, be = 0.0, gr = 0.0, gi = 0.0;
        for (int row = lane; row < p; row += 64) {
          const double2 x = ci[row], y = cj[row];
          al += x.x * x.x + x.y * x.y;
          be += y.x * y.x + y.y * y.y;
          const double2 g = cdotc(x, y);
          gr += g.x;
          gi += g.y;
        }
        al = fwave_sum(al);
        be = fwave_sum(be);
        gr = fwave_sum(gr);
        gi = fwave_sum(gi);
        const double g = hypot(gr, gi);
        if (!(al > 0.0 && be > 0.0 && g > tol * sqrt(al * be))) continue;
        const double2 e = make_double2(gr / g, gi / g);
        const double z = (be - al) / (2.0 * g);
        const double t = fabs(z) > 1e100 ? 0.5 / z : (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        const double2 se = make_double2(sn * e.x, sn * e.y);  // s e
        double2* vi = V + (int64_t)i * P;
        double2* vj = V + (int64_t)j * P;
        for (int row = lane; row < p; row += 64) {
          const double2 x = ci[row], y = cj[row];
          const double2 a1 = cdotc(se, y), b1 = cmul(se, x);  // s conj(e) y, s e x
          ci[row] = make_double2(cs * x.x - a1.x, cs * x.y - a1.y);
          cj[row] = make_double2(b1.x + cs * y.x, b1.y + cs * y.y);
          const double2 u = vi[row], v = vj[row];
          const double2 a2 = cdotc(se, v), b2 = cmul(se, u);
          vi[row] = make_double2(cs * u.x - a2.x, cs * u.y - a2.y);
          vj[row] = make_double2(b2.x + cs * v.x, b2.y + cs * v.y);
        }
        if (lane == 0) s_rot = 1;
      }
      __syncthreads();
    }
    conv = s_rot == 0;
    ++sweep;
    __syncthreads();
  }
  if (tid == 0) {
    st[4] = sweep;
    st[5] = conv ? 0 : 1;
  }
}

// Singular values (column norms of the rotated R2), their order, the rank rule of Alg. 2
// and the error figures.  One workgroup per matrix.
__global__ __launch_bounds__(kStepThreads) void k_fac_finish(FacWs ws, int32_t m, int32_t n, int32_t P, double eps,
                                                             double* __restrict__ sv, int32_t* __restrict__ rank,
                                                             int32_t* __restrict__ psteps, double* __restrict__ stats,
                                                             int32_t* __restrict__ status) {
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int32_t* st = ws.st(c);
  const int p = st[0];
  const double2* R = ws.R2(c);
  __shared__ double s_sig[kFacMaxP];
  __shared__ int s_ord[kFacMaxP];
  for (int i = wv; i < p; i += kStepThreads / 64) {
    double s = 0.0;
    for (int row = lane; row < p; row += 64) {
      const double2 v = R[(int64_t)i * P + row];
      s += v.x * v.x + v.y * v.y;
    }
    s = fwave_sum(s);
    if (lane == 0) s_sig[i] = sqrt(s);
  }
  __syncthreads();
  for (int i = tid; i < p; i += kStepThreads) {
    const double si = s_sig[i];
    int pos = 0;
    for (int j = 0; j < p; ++j) pos += (s_sig[j] > si || (s_sig[j] == si && j < i)) ? 1 : 0;
    s_ord[pos] = i;
  }
  __syncthreads();
  int32_t* ord = ws.ord(c);
  for (int t = tid; t < P; t += kStepThreads) {
    sv[(int64_t)c * P + t] = t < p ? s_sig[s_ord[t]] : 0.0;
    if (t < p) ord[t] = s_ord[t];
  }
  if (tid == 0) {
    const double smax = p > 0 ? s_sig[s_ord[0]] : 0.0;
    int l = 0;
    if (smax > 0.0)
      while (l < p && s_sig[s_ord[l]] > eps * smax) ++l;
    l = l < 1 ? 1 : l;
    const double T2 = ws.fro(c)[1];
    double tail2 = T2;
    for (int t = p - 1; t >= l; --t) tail2 += s_sig[s_ord[t]] * s_sig[s_ord[t]];
    // sigma_{l+1}(X) <= sqrt(sigma_{l+1}(B)^2 + T^2)
    const double sl = l < p ? s_sig[s_ord[l]] : 0.0;
    const double dropped = l < min(m, n) ? sqrt(sl * sl + T2) : 0.0;
    st[6] = l;
    rank[c] = l;
    psteps[c] = p;
    stats[3 * (int64_t)c] = sqrt(tail2);
    stats[3 * (int64_t)c + 1] = dropped;
    stats[3 * (int64_t)c + 2] = sqrt(T2);
    status[c] = (st[5] ? 2 : 0) | (st[7] ? 1 : 0);
  }
}

// The kept columns of J, in singular-value order, orthonormalised again by classical
// Gram-Schmidt applied twice; the result goes to the R2 area (R2 is no longer needed).
// One workgroup per matrix, rows tid and tid + 1024 per thread (p <= 2048).
__global__ __launch_bounds__(kBigThreads) void k_fac_orth(FacWs ws, int32_t P) {
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t* st = ws.st(c);
  const int p = st[0], l = st[6];
  const double2* J = ws.J(c);
  const int32_t* ord = ws.ord(c);
  double2* Q = ws.R2(c);
  __shared__ double2 s_v[kFacMaxP];
  __shared__ double2 s_h[kFacMaxP];
  __shared__ double s_red[kBigThreads / 64];
  if (p == 0) {  // a zero matrix: U = e_1
    for (int r = tid; r < P; r += kBigThreads) Q[r] = make_double2(r == 0 ? 1.0 : 0.0, 0.0);
    return;
  }
  const int r1 = tid + kBigThreads;
  for (int i = 0; i < l; ++i) {
    const double2* ji = J + (int64_t)ord[i] * P;
    double2 v = tid < p ? ji[tid] : make_double2(0.0, 0.0);
    double2 v1 = r1 < p ? ji[r1] : make_double2(0.0, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
      if (tid < p) s_v[tid] = v;
      if (r1 < p) s_v[r1] = v1;
      __syncthreads();
      for (int k = wv; k < i; k += kBigThreads / 64) {
        const double2* qk = Q + (int64_t)k * P;
        double hr = 0.0, hi = 0.0;
        for (int row = lane; row < p; row += 64) {
          const double2 t = cdotc(qk[row], s_v[row]);
          hr += t.x;
          hi += t.y;
        }
        hr = fwave_sum(hr);
        hi = fwave_sum(hi);
        if (lane == 0) s_h[k] = make_double2(hr, hi);
      }
      __syncthreads();
      if (tid < p) {
        for (int k = 0; k < i; ++k) {
          const double2 t = cmul(Q[(int64_t)k * P + tid], s_h[k]);
          v.x -= t.x;
          v.y -= t.y;
        }
      }
      if (r1 < p) {
        for (int k = 0; k < i; ++k) {
          const double2 t = cmul(Q[(int64_t)k * P + r1], s_h[k]);
          v1.x -= t.x;
          v1.y -= t.y;
        }
      }
      __syncthreads();
    }
    double s = fwave_sum(v.x * v.x + v.y * v.y + v1.x * v1.x + v1.y * v1.y);
    if (lane == 0) s_red[wv] = s;
    __syncthreads();
    double nrm2 = 0.0;
    for (int w = 0; w < kBigThreads / 64; ++w) nrm2 += s_red[w];
    const double inv = nrm2 > 0.0 ? 1.0 / sqrt(nrm2) : 0.0;
    if (tid < p) Q[(int64_t)i * P + tid] = make_double2(v.x * inv, v.y * inv);
    if (r1 < p) Q[(int64_t)i * P + r1] = make_double2(v1.x * inv, v1.y * inv);
    __syncthreads();
  }
}

// U = Q_p [Jo; 0]: the reflectors of the pivoted QR applied in reverse order to CPW = 16 /
// RPT kept columns per workgroup, held in registers (RPT rows per thread, rows tid + 1024 t).
template <int RPT>
__global__ __launch_bounds__(kBigThreads) void k_fac_u(FacWs ws, int32_t m, int32_t P, double2* __restrict__ U) {
  constexpr int CPW = 16 / RPT;
  constexpr int NW = kBigThreads / 64;
  const int c = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int32_t* st = ws.st(c);
  const int p = st[0], l = st[6];
  const int i0 = blockIdx.x * CPW;
  if (i0 >= l) return;
  const double2* Jo = ws.R2(c);
  __shared__ double2 s_d[2][NW][CPW];
  double2 z[CPW][RPT];
  const int prow = p > 0 ? p : 1;  // a zero matrix keeps e_1 in row 0
#pragma unroll
  for (int q = 0; q < CPW; ++q)
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int row = tid + kBigThreads * t;
      z[q][t] = (row < prow && i0 + q < l) ? Jo[(int64_t)(i0 + q) * P + row] : make_double2(0.0, 0.0);
    }
  const double2* Wm = ws.W(c);
  const double* omv = ws.om(c);
  for (int k = p - 1; k >= 0; --k) {
    const double2* w = Wm + (int64_t)k * m;
    const double om = omv[k];
    double2 wr[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int row = tid + kBigThreads * t;
      wr[t] = (row >= k && row < m) ? w[row] : make_double2(0.0, 0.0);
    }
    const int buf = k & 1;
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      double dr = 0.0, di = 0.0;
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const double2 v = cdotc(wr[t], z[q][t]);
        dr += v.x;
        di += v.y;
      }
      dr = fwave_sum(dr);
      di = fwave_sum(di);
      if (lane == 0) s_d[buf][wv][q] = make_double2(dr, di);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CPW; ++q) {
      double dr = 0.0, di = 0.0;
      for (int w2 = 0; w2 < NW; ++w2) {
        dr += s_d[buf][w2][q].x;
        di += s_d[buf][w2][q].y;
      }
      const double2 f = make_double2(om * dr, om * di);
#pragma unroll
      for (int t = 0; t < RPT; ++t) {
        const double2 fw = cmul(f, wr[t]);
        z[q][t].x -= fw.x;
        z[q][t].y -= fw.y;
      }
    }
  }
  double2* Um = U + (int64_t)c * m * P;
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    if (i0 + q >= l) break;
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int row = tid + kBigThreads * t;
      if (row < m) Um[(int64_t)(i0 + q) * m + row] = z[q][t];
    }
  }
}

// Sigma V^* = Jo^* B for the kept rows: SV[i][j] = conj(sum_k Jo[k][i] C[j][k]) (B = C^*),
// 16 x 16 output tiles staged through LDS.  Grid (ceil(n / 16), ceil(P / 16), batch).
constexpr int kSvT = 16;
__global__ __launch_bounds__(kSvT* kSvT) void k_fac_sv(FacWs ws, int32_t n, int32_t P, double2* __restrict__ SV) {
  const int c = blockIdx.z;
  const int32_t* st = ws.st(c);
  const int p = st[0], l = st[6];
  const int i0 = blockIdx.y * kSvT, j0 = blockIdx.x * kSvT;
  if (i0 >= l) return;
  const int ti = threadIdx.x % kSvT, tj = threadIdx.x / kSvT;
  const double2* Jo = ws.R2(c);
  const double2* C = ws.C(c);
  __shared__ double2 s_j[kSvT][kSvT + 1];  // [k][i]
  __shared__ double2 s_c[kSvT][kSvT + 1];  // [k][j]
  double ar = 0.0, ai = 0.0;
  for (int k0 = 0; k0 < p; k0 += kSvT) {
    {
      const int kk = threadIdx.x % kSvT, ii = threadIdx.x / kSvT;
      s_j[kk][ii] = (k0 + kk < p && i0 + ii < l) ? Jo[(int64_t)(i0 + ii) * P + k0 + kk] : make_double2(0.0, 0.0);
      const int jj = threadIdx.x % kSvT, k2 = threadIdx.x / kSvT;
      s_c[k2][jj] = (k0 + k2 < p && j0 + jj < n) ? C[(int64_t)(k0 + k2) * n + j0 + jj] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kSvT; ++kk) {
      const double2 t = cmul(s_j[kk][ti], s_c[kk][tj]);
      ar += t.x;
      ai += t.y;
    }
    __syncthreads();
  }
  const int i = i0 + ti, j = j0 + tj;
  if (i < l && j < n) SV[(int64_t)c * P * n + (int64_t)j * P + i] = make_double2(ar, -ai);
}

}  // namespace
}  // namespace uhm_detail

using namespace uhm_detail;

extern "C" {

int64_t uhm_cluster_basis_work(int32_t batch, int32_t m, int32_t n, int32_t pmax) {
  if (batch < 0 || m < 1 || n < 1 || pmax < 1) return -1;
  return layout(nullptr, m, n, pmax).per * (int64_t)batch;
}

int uhm_cluster_basis(double* X, int32_t batch, int32_t m, int32_t n, int32_t pmax, double tol, double eps,
                      double* U, double* SV, double* sv, int32_t* rank, int32_t* psteps, double* stats,
                      int32_t* status, double* work, int64_t work_len, void* hip_stream) {
  if (batch < 0 || m < 1 || n < 1) return fail(UHM_EINVAL, "uhm_cluster_basis: bad size");
  if (m > kFacMaxRows) return fail(UHM_EINVAL, "uhm_cluster_basis: more than 16384 rows");
  if (pmax < 1 || pmax > kFacMaxP || pmax > std::min(m, n))
    return fail(UHM_EINVAL, "uhm_cluster_basis: pmax must be in 1..min(m, n, 2048)");
  if (!(tol >= 0.0) || !std::isfinite(tol) || !(eps >= 0.0) || !std::isfinite(eps))
    return fail(UHM_EINVAL, "uhm_cluster_basis: tol and eps must be finite and >= 0");
  if (batch == 0) return UHM_OK;
  if (batch > 65535) return fail(UHM_EINVAL, "uhm_cluster_basis: more than 65535 matrices in one call");
  if (!X || !U || !SV || !sv || !rank || !psteps || !stats || !status || !work)
    return fail(UHM_EINVAL, "uhm_cluster_basis: null pointer");
  FacWs ws = layout(work, m, n, pmax);
  if (work_len < ws.per * (int64_t)batch) return fail(UHM_EINVAL, "uhm_cluster_basis: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  double2* Xc = reinterpret_cast<double2*>(X);
  UHM_HIP(hipMemsetAsync(work, 0, sizeof(double) * (size_t)(ws.per * (int64_t)batch), s));
  const int32_t P = pmax;
  const int32_t kcap = std::min(std::min(m, n), P);
  k_fac_norms<<<dim3((unsigned)((n + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(
      Xc, (int64_t)m * n, m, n, ws);
  UHM_HIP(hipGetLastError());
  QrStep q1{Xc, (int64_t)m * n, m, n, 0, kcap, tol * tol, 1, n, 1, 1};
  for (int32_t k = 0; k <= kcap; ++k) {
    k_qr_step<<<dim3((unsigned)((n + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(q1, ws,
                                                                                                              k);
    UHM_HIP(hipGetLastError());
  }
  // B^* (n x P, column-major) is in each matrix's C and Cq areas; the QR of the Cq copy gives R2
  FacWs wc = ws;
  double2* Cbase = ws.Cq(0);
  const int64_t c_stride = ws.per / 2;  // in complex elements
  k_fac_norms<<<dim3((unsigned)((P + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(
      Cbase, c_stride, n, P, wc);
  UHM_HIP(hipGetLastError());
  QrStep q2{Cbase, c_stride, n, P, 1, P, 0.0, 0, 1, P, 0};
  for (int32_t k = 0; k <= P; ++k) {
    k_qr_step<<<dim3((unsigned)((P + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(q2, ws,
                                                                                                              k);
    UHM_HIP(hipGetLastError());
  }
  const double jtol = std::sqrt((double)P) * 2.220446049250313e-16;
  k_fac_jacobi<<<dim3((unsigned)batch), dim3(kBigThreads), 0, s>>>(ws, P, jtol, 60);
  UHM_HIP(hipGetLastError());
  k_fac_finish<<<dim3((unsigned)batch), dim3(kStepThreads), 0, s>>>(ws, m, n, P, eps, sv, rank, psteps, stats, status);
  UHM_HIP(hipGetLastError());
  k_fac_orth<<<dim3((unsigned)batch), dim3(kBigThreads), 0, s>>>(ws, P);
  UHM_HIP(hipGetLastError());
  double2* Uc = reinterpret_cast<double2*>(U);
  const int rpt = (m + kBigThreads - 1) / kBigThreads;
#define UHM_FAC_U(R)                                                                                       \
  k_fac_u<R><<<dim3((unsigned)((P + 16 / R - 1) / (16 / R)), (unsigned)batch), dim3(kBigThreads), 0, s>>>( \
      ws, m, P, Uc)
  if (rpt <= 1)
    UHM_FAC_U(1);
  else if (rpt <= 2)
    UHM_FAC_U(2);
  else if (rpt <= 4)
    UHM_FAC_U(4);
  else if (rpt <= 8)
    UHM_FAC_U(8);
  else
    UHM_FAC_U(16);
#undef UHM_FAC_U
  UHM_HIP(hipGetLastError());
  k_fac_sv<<<dim3((unsigned)((n + kSvT - 1) / kSvT), (unsigned)((P + kSvT - 1) / kSvT), (unsigned)batch),
             dim3(kSvT * kSvT), 0, s>>>(ws, n, P, reinterpret_cast<double2*>(SV));
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

}  // extern "C"
