// Dense factorisations of the construction on the GPU, batched over matrices of one shape:
// Alg. 2's per-cluster SVD (section 4.2) and the algebraic recompression of ACA factors
// (section 2.3).
//
// Alg. 2.  For a cluster tau, Alg. 2 takes the SVD of the thin factor X_tau (n_tau x k_tau:
// the scaled left factors of the blocks in tau's block row) and keeps the left singular
// vectors whose singular values exceed eps * sigma_1.  They form U_tau, and U_tau^* X_tau =
// Sigma V^* gives the rows from which the couplings follow.  The SVD is taken in four steps:
//  1. Householder QR with column pivoting, X Pi = Q [R; 0] + (trailing part), stopped once
//     the trailing part's Frobenius norm T is at most tol * ||X||_F.  Then X = Q_p B + E with
//     B = R Pi^T = Q_p^* X (p x k) and E = (I - Q_p Q_p^*) X, ||E||_F = T.  The range of E is
//     orthogonal to that of Q_p, so X^* X = B^* B + E^* E and
//       sigma_i(B)^2 <= sigma_i(X)^2 <= sigma_i(B)^2 + T^2:
//     near the rank threshold eps sigma_1 a singular value moves by at most T^2 / (2 eps
//     sigma_1).  For the same reason the projection error of the basis U taken from B is
//     at most sqrt(sigma_{l+1}(X)^2 + T^2) in the 2-norm, and its Frobenius norm is exactly
//     sqrt(sum_{i>l} sigma_i(B)^2 + T^2).  With tol^2 about 1e-16 eps the rank test on B is
//     the one a full SVD of X takes, up to rounding.  One launch per step; every workgroup
//     of a matrix recomputes the pivot (largest remaining column norm, lowest index on ties)
//     and the trailing sum in the same order, so all of them take the same decisions.
//     Columns are never moved: a pivot column is retired (norm marker -1) and R is kept in
//     the original column order, which is B itself.
//  2. Unpivoted Householder QR of B^* = Q2 R2, R2 p x p (the same step kernel).
//  3. One-sided (Hestenes) Jacobi on the columns of M = R2^*: M J = W Sigma, and since
//     B = R2^* Q2^* = M Q2^*, the left singular vectors of B are the columns of W, which are
//     the rotated columns scaled by 1 / sigma_i (the column norms); the rotations J are not
//     kept.  A rotated column carries an absolute error of about eps_mach sigma_1, so the
//     direction of w_i is off by about eps_mach sigma_1 / sigma_i, and its share of the
//     projection error stays at eps_mach sigma_1.  Round-robin pairs: one launch per round
//     over the whole batch, one wavefront per pair, and one read-back per sweep.  The kept
//     columns are orthonormalised (classical Gram-Schmidt applied twice, largest singular
//     value first) into W_l.
//  4. U = Q_p [W_l; 0] (the reflectors of step 1 applied in reverse order, the columns held
//     in registers) and Sigma V^* = W_l^* B.
//
// Recompression.  A block A|_b ~ X Y^* from ACA (k terms) is brought to its SVD truncated at
// eps sigma_1: unpivoted QR of both factors, X = Q_X R_X and Y = Q_Y R_Y; one-sided Jacobi
// on M = R_Y R_X^*, M J = W Sigma (the columns of W come out orthogonal relative to their
// own norms, whatever those are), so X Y^* = Q_X M^* Q_Y^* = (Q_X J) Sigma (Q_Y W)^*; the
// kept columns of J and of W are orthonormalised again as above and carried back through
// the reflectors.
#include "uhm_internal.h"

#include <climits>
#include <cmath>

namespace uhm_detail {
namespace {

constexpr int kFacMaxP = 2048;      // largest Jacobi order
constexpr int kFacMaxRows = 16384;  // largest row count: 16 rows per thread in the apply kernel
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

// One array per matrix of the batch: matrix c's array starts at p + c * stride.
template <class T>
struct Arr {
  T* p;
  int64_t stride;
  __host__ __device__ T* at(int c) const { return p + (int64_t)c * stride; }
};
using CArr = Arr<double2>;
using DArr = Arr<double>;
using IArr = Arr<int32_t>;

// Workspace: each matrix owns `per` doubles; regions are carved out in 256-byte units.
struct Carve {
  int64_t per = 0;
  int64_t take(int64_t doubles) {
    const int64_t o = per;
    per += (doubles + 31) / 32 * 32;
    return o;
  }
};
template <class T>
Arr<T> region(double* base, int64_t per, int64_t off) {
  return Arr<T>{reinterpret_cast<T*>(base + off), (int64_t)(per * sizeof(double) / sizeof(T))};
}

// Squared column norms of a rows x cols matrix (lda = rows) into nu's first buffer: one
// wavefront per column, kStepCols columns per workgroup.  A zero column is marked retired
// (-1) at once: its R entries are zero and the QR steps leave it alone.
__global__ __launch_bounds__(kStepThreads) void k_col_norms(CArr A, int32_t rows, int32_t cols, DArr nu) {
  const int c = blockIdx.y;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double2* Am = A.at(c);
  double* nm = nu.at(c);
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
    if (lane == 0) nm[j] = s > 0.0 ? s : -1.0;
  }
}

struct QrStep {
  CArr A;  // rows x cols per matrix, column-major (lda = rows), updated in place
  int32_t rows, cols;
  DArr nu;   // 2 * cols squared column norms (double-buffered by step parity)
  CArr W;    // reflector k at W + k * rows (W.p null: not kept)
  DArr om;   // omega_k
  CArr R;    // R[k][j] at R[k * rs + j * cs], conjugated if rconj
  CArr Rq;   // a second copy of R (Rq.p may be null)
  int32_t rs, cs, rconj;
  IArr st;   // [0] steps taken, [1] stopped, [2] the step cap came before the tolerance
  IArr lim;  // per-matrix step limit at lim.at(c)[0] (lim.p null: none)
  DArr fro;  // pivoted: [0] ||A||_F^2, [1] T^2 (the trailing sum at the stop)
  int32_t kcap;
  double tol2;  // pivoted: stop when T^2 <= tol2 * ||A||_F^2
  int32_t pivoted;
};

// The reflector of step k is P = I - omega w w^*, w = x - beta e_k on rows k.., x the pivot
// column, beta = -e^{i arg x_k} ||x|| (so that w_k carries no cancellation), omega =
// 1 / (||x|| (||x|| + |x_k|)); P x = beta e_k.
struct StepHead {
  int piv;
  double2 beta, wk;
  double om;
};

// The part of a step every workgroup of a matrix takes alike: the trailing sum and the
// pivot over the live columns (reduced in one fixed order), the stop test, and the
// reflector.  Returns false when the matrix has stopped (in this step or before).
template <int NT>
__device__ bool qr_head(const QrStep& a, int32_t k, int c, StepHead& h) {
  __shared__ double s_sum[NT], s_mx[NT];
  __shared__ int s_ix[NT];
  int32_t* st = a.st.at(c);
  if (st[1]) return false;  // stopped in an earlier step
  const int tid = threadIdx.x;
  const double* nu = a.nu.at(c) + (k & 1) * (int64_t)a.cols;
  const int32_t lim = a.lim.p ? min(a.kcap, a.lim.at(c)[0]) : a.kcap;
  double sum = 0.0, mx = -1.0;
  int ix = INT_MAX;
  for (int j = tid; j < a.cols; j += NT) {
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
  for (int s = NT / 2; s > 0; s >>= 1) {
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
  double* fro = a.pivoted ? a.fro.at(c) : nullptr;
  const double f2 = k == 0 || !fro ? tr : fro[0];
  const bool met = a.pivoted && (tr <= a.tol2 * f2 || s_mx[0] <= 0.0);
  if (k >= lim || k >= a.rows || met) {
    if (blockIdx.x == 0 && tid == 0) {
      st[0] = k;
      st[1] = 1;
      if (fro) {
        fro[0] = f2;
        fro[1] = tr;
      }
      st[2] = a.pivoted && !met && k < a.rows && k < a.cols ? 1 : 0;
    }
    return false;
  }
  if (fro && k == 0 && blockIdx.x == 0 && tid == 0) fro[0] = tr;
  h.piv = a.pivoted ? s_ix[0] : k;
  const double2* x = a.A.at(c) + (int64_t)h.piv * a.rows;
  const double nx = sqrt(fmax(nu[h.piv], 0.0));
  const double2 al = x[k];
  const double aa = hypot(al.x, al.y);
  const double2 ph = aa > 0.0 ? make_double2(al.x / aa, al.y / aa) : make_double2(1.0, 0.0);
  h.beta = make_double2(-ph.x * nx, -ph.y * nx);
  h.wk = make_double2(ph.x * (aa + nx), ph.y * (aa + nx));
  h.om = nx > 0.0 ? 1.0 / (nx * (nx + aa)) : 0.0;
  return true;
}

// The pivot column's part of a step (its reflector, R entry and retired marker), and the
// R entry and marker of a column retired before; `lead` is the one thread that writes the
// scalars.  The reflector is written by the threads t = 0..NT-1 of the caller.
__device__ __forceinline__ void qr_retire(const QrStep& a, int32_t k, int c, const StepHead& h, int j, bool lead,
                                          int t0, int nt) {
  const int64_t ro = (int64_t)k * a.rs + (int64_t)j * a.cs;
  double* nu2 = a.nu.at(c) + ((k + 1) & 1) * (int64_t)a.cols;
  double2* R = a.R.at(c);
  double2* Rq = a.Rq.p ? a.Rq.at(c) : nullptr;
  if (j == h.piv) {
    if (a.W.p) {
      const double2* x = a.A.at(c) + (int64_t)h.piv * a.rows;
      double2* w = a.W.at(c) + (int64_t)k * a.rows;
      for (int i = t0; i < a.rows; i += nt) w[i] = i < k ? make_double2(0.0, 0.0) : (i == k ? h.wk : x[i]);
      if (lead) a.om.at(c)[k] = h.om;
    }
    if (lead) {
      R[ro] = a.rconj ? cconj(h.beta) : h.beta;
      if (Rq) Rq[ro] = R[ro];
      nu2[j] = -1.0;
    }
  } else if (lead) {  // retired in an earlier step: R is upper triangular in pivot order
    R[ro] = make_double2(0.0, 0.0);
    if (Rq) Rq[ro] = make_double2(0.0, 0.0);
    nu2[j] = -1.0;
  }
}

__device__ __forceinline__ void qr_store(const QrStep& a, int32_t k, int c, int j, double2 rk, double nn) {
  const int64_t ro = (int64_t)k * a.rs + (int64_t)j * a.cs;
  double2* R = a.R.at(c);
  R[ro] = a.rconj ? cconj(rk) : rk;
  if (a.Rq.p) a.Rq.at(c)[ro] = R[ro];
  a.nu.at(c)[((k + 1) & 1) * (int64_t)a.cols + j] = nn;
}

// One Householder step k for every matrix of the batch, matrices of at most 64 * RPL rows:
// a wavefront per column, kStepCols columns per workgroup, grid (ceil(cols / 16), batch).
// The pivot column (once per wavefront) and each updated column are held in registers (RPL
// rows per lane), so a column is read once and written once.
template <int RPL>
__global__ __launch_bounds__(kStepThreads) void k_qr_step(QrStep a, int32_t k) {
  const int c = blockIdx.y;
  StepHead h;
  if (!qr_head<kStepThreads>(a, k, c, h)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double* nu = a.nu.at(c) + (k & 1) * (int64_t)a.cols;
  double2* Am = a.A.at(c);
  const double2* x = Am + (int64_t)h.piv * a.rows;
  double2 xc[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = k + lane + 64 * t;
    xc[t] = i < a.rows ? (i == k ? h.wk : x[i]) : make_double2(0.0, 0.0);
  }
  for (int q = 0; q < kStepCols / 4; ++q) {
    const int j = blockIdx.x * kStepCols + wv * (kStepCols / 4) + q;
    if (j >= a.cols) break;
    if (j == h.piv || nu[j] < 0.0) {
      qr_retire(a, k, c, h, j, lane == 0, lane, 64);
      continue;
    }
    double2* y = Am + (int64_t)j * a.rows;
    double2 yc[RPL];
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = k + lane + 64 * t;
      yc[t] = i < a.rows ? y[i] : make_double2(0.0, 0.0);
      const double2 v = cdotc(xc[t], yc[t]);
      sr += v.x;
      si += v.y;
    }
    sr = fwave_sum(sr);
    si = fwave_sum(si);
    const double2 f = make_double2(h.om * sr, h.om * si);
    double nn = 0.0;
    double2 rk = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = k + lane + 64 * t;
      if (i < a.rows) {
        const double2 fw = cmul(f, xc[t]);
        const double2 v = make_double2(yc[t].x - fw.x, yc[t].y - fw.y);
        y[i] = v;
        if (i == k)
          rk = v;
        else
          nn += v.x * v.x + v.y * v.y;
      }
    }
    nn = fwave_sum(nn);
    if (lane == 0) qr_store(a, k, c, j, rk, nn);  // lane 0 holds row k
  }
}

// The same step for matrices of more rows: a workgroup of NT threads per column (RPL rows
// per thread, rows k + tid + NT t), kWideCols columns per workgroup in turn, the partial
// sums of the NT / 64 wavefronts combined in LDS in one fixed order.
constexpr int kWideCols = 8;
template <int NT, int RPL>
__global__ __launch_bounds__(NT) void k_qr_step_wide(QrStep a, int32_t k) {
  constexpr int NW = NT / 64;
  const int c = blockIdx.y;
  StepHead h;
  if (!qr_head<NT>(a, k, c, h)) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  __shared__ double s_a[2][NW], s_b[2][NW];
  const double* nu = a.nu.at(c) + (k & 1) * (int64_t)a.cols;
  double2* Am = a.A.at(c);
  const double2* x = Am + (int64_t)h.piv * a.rows;
  double2 xc[RPL];
#pragma unroll
  for (int t = 0; t < RPL; ++t) {
    const int i = k + tid + NT * t;
    xc[t] = i < a.rows ? (i == k ? h.wk : x[i]) : make_double2(0.0, 0.0);
  }
  for (int q = 0; q < kWideCols; ++q) {
    const int j = blockIdx.x * kWideCols + q;
    if (j >= a.cols) break;
    if (j == h.piv || nu[j] < 0.0) {
      qr_retire(a, k, c, h, j, tid == 0, tid, NT);
      continue;
    }
    double2* y = Am + (int64_t)j * a.rows;
    double2 yc[RPL];
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = k + tid + NT * t;
      yc[t] = i < a.rows ? y[i] : make_double2(0.0, 0.0);
      const double2 v = cdotc(xc[t], yc[t]);
      sr += v.x;
      si += v.y;
    }
    sr = fwave_sum(sr);
    si = fwave_sum(si);
    const int b = q & 1;
    if (lane == 0) {
      s_a[b][wv] = sr;
      s_b[b][wv] = si;
    }
    __syncthreads();
    sr = 0.0;
    si = 0.0;
    for (int w = 0; w < NW; ++w) {
      sr += s_a[b][w];
      si += s_b[b][w];
    }
    const double2 f = make_double2(h.om * sr, h.om * si);
    double nn = 0.0;
    double2 rk = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int i = k + tid + NT * t;
      if (i < a.rows) {
        const double2 fw = cmul(f, xc[t]);
        const double2 v = make_double2(yc[t].x - fw.x, yc[t].y - fw.y);
        y[i] = v;
        if (i == k)
          rk = v;
        else
          nn += v.x * v.x + v.y * v.y;
      }
    }
    nn = fwave_sum(nn);
    __syncthreads();  // every wavefront has read s_a[b] before it is written again
    if (lane == 0) s_a[b][wv] = nn;
    __syncthreads();
    if (tid == 0) {  // thread 0 holds row k
      double t2 = 0.0;
      for (int w = 0; w < NW; ++w) t2 += s_a[b][w];
      qr_store(a, k, c, j, rk, t2);
    }
  }
}

// One-sided Jacobi on the p x p matrix R (ld P; p = pp.at(c)[0]), the rotations accumulated
// in V unless V is null.  A sweep is P' - 1 rounds (P' = P rounded up to even) of the circle schedule: index 0
// fixed, the others rotated, so the pairs of a round are disjoint; each round is one launch
// over the whole batch, one wavefront per pair, and pairs with a column >= p are skipped.
// A pair (i, j) with Gram entries alpha, beta, gamma is rotated when |gamma| > tol
// sqrt(alpha beta): with e = gamma / |gamma|, zeta = (beta - alpha) / (2 |gamma|) and t the
// smaller root of t^2 + 2 zeta t - 1 = 0, c = 1 / sqrt(1 + t^2), s = c t,
//   a_i <- c a_i - s conj(e) a_j,   a_j <- s e a_i + c a_j,
// which makes a_i^* a_j vanish.  sst per matrix: [0] a rotation in this sweep, [1] sweeps,
// [2] still running (not converged), [3] rank (written later).
constexpr int kJacWaves = 4;

__global__ __launch_bounds__(256) void k_jacobi_init(CArr Va, int32_t P, IArr pp, IArr sst) {
  const int c = blockIdx.y;
  const int p = pp.at(c)[0];
  if (Va.p) {  // no accumulator: the rotations are not kept
    double2* V = Va.at(c);
    for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < (int64_t)P * P; q += (int64_t)gridDim.x * 256) {
      const int r = (int)(q % P), col = (int)(q / P);
      V[q] = make_double2(r == col && r < p ? 1.0 : 0.0, 0.0);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int32_t* t = sst.at(c);
    t[0] = 0;
    t[1] = 0;
    t[2] = p >= 2 ? 1 : 0;
  }
}

// Round r of the circle schedule over ns + (ns & 1) indices (ns >= every matrix's p; R and V
// have leading dimension P).
__global__ __launch_bounds__(64 * kJacWaves) void k_jacobi_round(CArr Ra, CArr Va, int32_t P, int32_t ns, IArr pp,
                                                                 IArr sst, int32_t r, double tol) {
  const int c = blockIdx.y;
  int32_t* t = sst.at(c);
  if (!t[2]) return;
  const int lane = threadIdx.x & 63;
  const int q = blockIdx.x * kJacWaves + (threadIdx.x >> 6);
  const int pq = ns + (ns & 1);
  if (q >= pq / 2) return;
  const int p = pp.at(c)[0];
  const int a0 = q == 0 ? 0 : (r + q - 1) % (pq - 1) + 1;
  const int b0 = (r + (pq - 1 - q) - 1) % (pq - 1) + 1;
  const int i = min(a0, b0), j = max(a0, b0);
  if (j >= p) return;
  double2* R = Ra.at(c);
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
  if (!(al > 0.0 && be > 0.0 && g > tol * sqrt(al * be))) return;
  const double2 e = make_double2(gr / g, gi / g);
  const double z = (be - al) / (2.0 * g);
  const double tt = fabs(z) > 1e100 ? 0.5 / z : (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
  const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
  const double2 se = make_double2(sn * e.x, sn * e.y);  // s e
  for (int row = lane; row < p; row += 64) {
    const double2 x = ci[row], y = cj[row];
    const double2 a1 = cdotc(se, y), b1 = cmul(se, x);  // s conj(e) y, s e x
    ci[row] = make_double2(cs * x.x - a1.x, cs * x.y - a1.y);
    cj[row] = make_double2(b1.x + cs * y.x, b1.y + cs * y.y);
  }
  if (Va.p) {
    double2* vi = Va.at(c) + (int64_t)i * P;
    double2* vj = Va.at(c) + (int64_t)j * P;
    for (int row = lane; row < p; row += 64) {
      const double2 u = vi[row], v = vj[row];
      const double2 a2 = cdotc(se, v), b2 = cmul(se, u);
      vi[row] = make_double2(cs * u.x - a2.x, cs * u.y - a2.y);
      vj[row] = make_double2(b2.x + cs * v.x, b2.y + cs * v.y);
    }
  }
  if (lane == 0) t[0] = 1;
}

// The largest value of v.at(c)[0] over the batch, into *out (set to 0 before).
__global__ __launch_bounds__(256) void k_batch_max(IArr v, int32_t batch, int32_t* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c < batch) atomicMax(out, v.at(c)[0]);
}

// End of a sweep: a matrix with no rotation in it has converged; the rest are counted.
__global__ __launch_bounds__(256) void k_jacobi_sweep_end(IArr sst, int32_t batch, int32_t* __restrict__ active) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= batch) return;
  int32_t* t = sst.at(c);
  if (t[2]) {
    t[1] += 1;
    if (!t[0])
      t[2] = 0;
    else
      atomicAdd(active, 1);
  }
  t[0] = 0;
}

// Orders up to 64: one workgroup per matrix keeps R and V in LDS (2 x 64 KB) through all
// sweeps, the pairs of a round taken by its 8 wavefronts and the rounds separated by
// barriers; the schedule is the same circle over p + (p & 1) indices.
constexpr int kJacLds = 64;
__global__ __launch_bounds__(512) void k_jacobi_lds(CArr Ra, CArr Va, int32_t P, IArr pp, IArr sst, double tol,
                                                    int32_t max_sweeps) {
  __shared__ double2 sR[kJacLds * kJacLds];
  __shared__ double2 sV[kJacLds * kJacLds];
  __shared__ int s_rot;
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int p = pp.at(c)[0];
  const bool acc = Va.p != nullptr;  // accumulate the rotations in V
  double2* R = Ra.at(c);
  for (int q = tid; q < P * P; q += 512) {
    const int r = q % P, col = q / P;
    sR[r + col * kJacLds] = R[q];
    sV[r + col * kJacLds] = make_double2(r == col && r < p ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  const int pq = p + (p & 1);
  int sweep = 0;
  bool conv = p < 2;
  while (!conv && sweep < max_sweeps) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < pq - 1; ++r) {
      for (int q = wv; q < pq / 2; q += 8) {
        const int a0 = q == 0 ? 0 : (r + q - 1) % (pq - 1) + 1;
        const int b0 = (r + (pq - 1 - q) - 1) % (pq - 1) + 1;
        const int i = min(a0, b0), j = max(a0, b0);
        if (j >= p) continue;
        double2* ci = sR + i * kJacLds;
        double2* cj = sR + j * kJacLds;
        const double2 x = lane < p ? ci[lane] : make_double2(0.0, 0.0);
        const double2 y = lane < p ? cj[lane] : make_double2(0.0, 0.0);
        const double2 gg = cdotc(x, y);
        const double al = fwave_sum(x.x * x.x + x.y * x.y);
        const double be = fwave_sum(y.x * y.x + y.y * y.y);
        const double gr = fwave_sum(gg.x), gi = fwave_sum(gg.y);
        const double g = hypot(gr, gi);
        if (!(al > 0.0 && be > 0.0 && g > tol * sqrt(al * be))) continue;
        const double2 e = make_double2(gr / g, gi / g);
        const double z = (be - al) / (2.0 * g);
        const double tt = fabs(z) > 1e100 ? 0.5 / z : (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
        const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        const double2 se = make_double2(sn * e.x, sn * e.y);  // s e
        if (lane < p) {
          const double2 a1 = cdotc(se, y), b1 = cmul(se, x);
          ci[lane] = make_double2(cs * x.x - a1.x, cs * x.y - a1.y);
          cj[lane] = make_double2(b1.x + cs * y.x, b1.y + cs * y.y);
        }
        if (acc && lane < p) {
          double2* vi = sV + i * kJacLds;
          double2* vj = sV + j * kJacLds;
          const double2 u = vi[lane], v = vj[lane];
          const double2 a2 = cdotc(se, v), b2 = cmul(se, u);
          vi[lane] = make_double2(cs * u.x - a2.x, cs * u.y - a2.y);
          vj[lane] = make_double2(b2.x + cs * v.x, b2.y + cs * v.y);
        }
        if (lane == 0) s_rot = 1;
      }
      __syncthreads();
    }
    conv = s_rot == 0;
    ++sweep;
    __syncthreads();
  }
  for (int q = tid; q < P * P; q += 512) {
    const int r = q % P, col = q / P;
    R[q] = sR[r + col * kJacLds];
    if (acc) Va.at(c)[q] = sV[r + col * kJacLds];
  }
  if (tid == 0) {
    int32_t* t = sst.at(c);
    t[0] = 0;
    t[1] = sweep;
    t[2] = conv ? 0 : 1;
  }
}

// The sweeps of one batch: one launch per round, and the count of running matrices read back
// after each sweep (active: one device int); orders up to 64 in LDS, one launch in all.  ns:
// the largest order in the batch (the round schedule's size); P: the leading dimension.
int run_jacobi(CArr R, CArr V, int32_t P, int32_t ns, IArr pp, IArr sst, int32_t batch, double tol,
               int32_t max_sweeps, int32_t* active, hipStream_t s) {
  if (P <= kJacLds) {
    k_jacobi_lds<<<dim3((unsigned)batch), dim3(512), 0, s>>>(R, V, P, pp, sst, tol, max_sweeps);
    UHM_HIP(hipGetLastError());
    return UHM_OK;
  }
  const int64_t pq = ns + (ns & 1);
  const unsigned gx = (unsigned)std::min<int64_t>(((int64_t)P * P + 255) / 256, 1024);
  k_jacobi_init<<<dim3(gx, (unsigned)batch), dim3(256), 0, s>>>(V, P, pp, sst);
  UHM_HIP(hipGetLastError());
  const unsigned rx = (unsigned)((pq / 2 + kJacWaves - 1) / kJacWaves);
  for (int32_t sweep = 0; sweep < max_sweeps && pq >= 2; ++sweep) {
    for (int32_t r = 0; r < pq - 1; ++r) {
      k_jacobi_round<<<dim3(rx, (unsigned)batch), dim3(64 * kJacWaves), 0, s>>>(R, V, P, ns, pp, sst, r, tol);
      UHM_HIP(hipGetLastError());
    }
    UHM_HIP(hipMemsetAsync(active, 0, sizeof(int32_t), s));
    k_jacobi_sweep_end<<<dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s>>>(sst, batch, active);
    UHM_HIP(hipGetLastError());
    int32_t left = 0;
    UHM_HIP(hipMemcpyAsync(&left, active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    UHM_HIP(hipStreamSynchronize(s));
    if (left == 0) break;
  }
  return UHM_OK;
}

struct Finish {
  CArr R;  // the rotated matrix (ld P); singular values are its column norms
  int32_t P;
  IArr pp;          // p at pp.at(c)[0]
  IArr sst;         // [2] Jacobi not converged (read), [3] rank l (written)
  IArr ord;         // P ints: columns in singular-value order (written)
  double eps;       // rank rule: sigma > eps * sigma_1, at least 1
  DArr fro;         // T^2 at fro.at(c)[1] (fro.p null: 0)
  IArr qst;         // the pivoted QR's state, [2] = step cap first (qst.p null: none)
  int32_t m, n;     // shape, for the dropped value
  double* sv;       // P per matrix
  int32_t* rank;
  int32_t* psteps;  // may be null
  double* stats;    // 3 per matrix, may be null
  int32_t* status;
};

// Singular values (column norms of the rotated matrix), their order, the rank rule and the
// error figures.  One workgroup per matrix.
__global__ __launch_bounds__(kStepThreads) void k_finish(Finish f) {
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int p = f.pp.at(c)[0];
  const double2* R = f.R.at(c);
  __shared__ double s_sig[kFacMaxP];
  __shared__ int s_ord[kFacMaxP];
  for (int i = wv; i < p; i += kStepThreads / 64) {
    double s = 0.0;
    for (int row = lane; row < p; row += 64) {
      const double2 v = R[(int64_t)i * f.P + row];
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
  int32_t* ord = f.ord.at(c);
  for (int t = tid; t < f.P; t += kStepThreads) {
    f.sv[(int64_t)c * f.P + t] = t < p ? s_sig[s_ord[t]] : 0.0;
    if (t < p) ord[t] = s_ord[t];
  }
  if (tid == 0) {
    const double smax = p > 0 ? s_sig[s_ord[0]] : 0.0;
    int l = 0;
    if (smax > 0.0)
      while (l < p && s_sig[s_ord[l]] > f.eps * smax) ++l;
    l = l < 1 ? 1 : l;
    f.sst.at(c)[3] = l;
    f.rank[c] = l;
    if (f.psteps) f.psteps[c] = p;
    if (f.stats) {
      const double T2 = f.fro.p ? f.fro.at(c)[1] : 0.0;
      double tail2 = T2;
      for (int t = p - 1; t >= l; --t) tail2 += s_sig[s_ord[t]] * s_sig[s_ord[t]];
      // sigma_{l+1}(X) <= sqrt(sigma_{l+1}(B)^2 + T^2)
      const double sl = l < p ? s_sig[s_ord[l]] : 0.0;
      f.stats[3 * (int64_t)c] = sqrt(tail2);
      f.stats[3 * (int64_t)c + 1] = l < min(f.m, f.n) ? sqrt(sl * sl + T2) : 0.0;
      f.stats[3 * (int64_t)c + 2] = sqrt(T2);
    }
    const int cap = f.qst.p ? f.qst.at(c)[2] : 0;
    f.status[c] = (f.sst.at(c)[2] ? 2 : 0) | (cap ? 1 : 0);
  }
}

// Columns ord[0..l) of src (p rows, ld lds) orthonormalised by classical Gram-Schmidt
// applied twice, in that order, into dst (ld ldd).  One workgroup per matrix, rows tid and
// tid + 1024 per thread (p <= 2048).  A zero matrix (p = 0) gives e_1.
__global__ __launch_bounds__(kBigThreads) void k_orth(CArr src, int32_t lds, IArr ord_a, IArr pp, IArr sst, CArr dst,
                                                      int32_t ldd) {
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int p = pp.at(c)[0], l = sst.at(c)[3];
  const double2* J = src.at(c);
  const int32_t* ord = ord_a.at(c);
  double2* Q = dst.at(c);
  __shared__ double2 s_v[kFacMaxP];
  __shared__ double2 s_h[kFacMaxP];
  __shared__ double s_red[kBigThreads / 64];
  if (p == 0) {
    if (tid == 0) Q[0] = make_double2(1.0, 0.0);
    return;
  }
  const int r1 = tid + kBigThreads;
  for (int i = 0; i < l; ++i) {
    const double2* ji = J + (int64_t)ord[i] * lds;
    double2 v = tid < p ? ji[tid] : make_double2(0.0, 0.0);
    double2 v1 = r1 < p ? ji[r1] : make_double2(0.0, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
      if (tid < p) s_v[tid] = v;
      if (r1 < p) s_v[r1] = v1;
      __syncthreads();
      for (int k = wv; k < i; k += kBigThreads / 64) {
        const double2* qk = Q + (int64_t)k * ldd;
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
          const double2 t = cmul(Q[(int64_t)k * ldd + tid], s_h[k]);
          v.x -= t.x;
          v.y -= t.y;
        }
      }
      if (r1 < p) {
        for (int k = 0; k < i; ++k) {
          const double2 t = cmul(Q[(int64_t)k * ldd + r1], s_h[k]);
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
    if (tid < p) Q[(int64_t)i * ldd + tid] = make_double2(v.x * inv, v.y * inv);
    if (r1 < p) Q[(int64_t)i * ldd + r1] = make_double2(v1.x * inv, v1.y * inv);
    __syncthreads();
  }
}

struct Apply {
  CArr W;       // reflector k at W + k * rows
  DArr om;
  int32_t rows;
  IArr nref;    // reflectors at nref.at(c)[0]
  CArr src;     // kept columns, rows 0..p-1 (p at pp.at(c)[0], at least 1), ld lds
  int32_t lds;
  IArr pp;
  IArr sst;     // l at sst.at(c)[3]
  CArr dst;     // rows x l, ld rows
};

// dst = Q [src; 0] with Q = P_0 P_1 ... the reflectors applied in reverse order, CPW = 16 /
// RPT kept columns per workgroup of NT threads held in registers (RPT rows per thread, rows
// tid + NT t).
template <int RPT, int NT>
__global__ __launch_bounds__(NT) void k_apply_q(Apply a) {
  constexpr int CPW = 16 / RPT;
  constexpr int NW = NT / 64;
  const int c = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nr = a.nref.at(c)[0], l = a.sst.at(c)[3];
  const int p = a.pp.at(c)[0] > 0 ? a.pp.at(c)[0] : 1;  // a zero matrix keeps e_1 in row 0
  const int i0 = blockIdx.x * CPW;
  if (i0 >= l) return;
  const double2* S = a.src.at(c);
  __shared__ double2 s_d[2][NW][CPW];
  double2 z[CPW][RPT];
#pragma unroll
  for (int q = 0; q < CPW; ++q)
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int row = tid + NT * t;
      z[q][t] = (row < p && i0 + q < l) ? S[(int64_t)(i0 + q) * a.lds + row] : make_double2(0.0, 0.0);
    }
  const double2* Wm = a.W.at(c);
  const double* omv = a.om.at(c);
  for (int k = nr - 1; k >= 0; --k) {
    const double2* w = Wm + (int64_t)k * a.rows;
    const double om = omv[k];
    double2 wr[RPT];
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int row = tid + NT * t;
      wr[t] = (row >= k && row < a.rows) ? w[row] : make_double2(0.0, 0.0);
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
  double2* D = a.dst.at(c);
#pragma unroll
  for (int q = 0; q < CPW; ++q) {
    if (i0 + q >= l) break;
#pragma unroll
    for (int t = 0; t < RPT; ++t) {
      const int row = tid + NT * t;
      if (row < a.rows) D[(int64_t)(i0 + q) * a.rows + row] = z[q][t];
    }
  }
}

int launch_apply(const Apply& a, int32_t colcap, int32_t batch, hipStream_t s) {
  const int rpt = (a.rows + kBigThreads - 1) / kBigThreads;
#define UHM_APPLY(R, T)                                                                                  \
  k_apply_q<R, T><<<dim3((unsigned)((colcap + 16 / R - 1) / (16 / R)), (unsigned)batch), dim3(T), 0, s>>>(a)
  if (a.rows <= 64)
    UHM_APPLY(1, 64);
  else if (a.rows <= 128)
    UHM_APPLY(1, 128);
  else if (a.rows <= 256)
    UHM_APPLY(1, 256);
  else if (a.rows <= 512)
    UHM_APPLY(1, 512);
  else if (rpt <= 1)
    UHM_APPLY(1, 1024);
  else if (rpt <= 2)
    UHM_APPLY(2, 1024);
  else if (rpt <= 4)
    UHM_APPLY(4, 1024);
  else if (rpt <= 8)
    UHM_APPLY(8, 1024);
  else
    UHM_APPLY(16, 1024);
#undef UHM_APPLY
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

// Sigma V^* = Jo^* B for the kept rows: SV[i][j] = conj(sum_k Jo[k][i] C[j][k]) (B = C^*),
// 16 x 16 output tiles staged through LDS.  Grid (ceil(n / 16), ceil(P / 16), batch).
constexpr int kSvT = 16;
__global__ __launch_bounds__(kSvT* kSvT) void k_fac_sv(CArr Joa, int32_t P, IArr pp, IArr sst, CArr Ca, int32_t n,
                                                       double2* __restrict__ SV) {
  const int c = blockIdx.z;
  const int p = pp.at(c)[0], l = sst.at(c)[3];
  const int i0 = blockIdx.y * kSvT, j0 = blockIdx.x * kSvT;
  if (i0 >= l) return;
  const int ti = threadIdx.x % kSvT, tj = threadIdx.x / kSvT;
  const double2* Jo = Joa.at(c);
  const double2* C = Ca.at(c);
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

// M = R_Y R_X^* (kp x kp; both upper triangular, ld kp): M[i][j] = sum_{l >= max(i, j)}
// R_Y[i][l] conj(R_X[j][l]).  Grid (ceil(kp / 16), ceil(kp / 16), batch), one thread per entry.
__global__ __launch_bounds__(256) void k_rr(CArr RYa, CArr RXa, int32_t kp, CArr Ma) {
  const int c = blockIdx.z;
  const int i = blockIdx.y * 16 + threadIdx.x % 16, j = blockIdx.x * 16 + threadIdx.x / 16;
  if (i >= kp || j >= kp) return;
  const double2* RY = RYa.at(c);
  const double2* RX = RXa.at(c);
  double ar = 0.0, ai = 0.0;
  for (int l = max(i, j); l < kp; ++l) {
    const double2 t = cdotc(RX[j + (int64_t)l * kp], RY[i + (int64_t)l * kp]);
    ar += t.x;
    ai += t.y;
  }
  Ma.at(c)[i + (int64_t)j * kp] = make_double2(ar, ai);
}

// The couplings of the construction, one workgroup per admissible block b = (tau, sigma):
// S_{X,b} = L_{tau,b} Sigma_b^{-1} (l_tau x k_b), S_{Y,b} = conj(L_{sigma,b}) (l_sigma x k_b) and
// S_b = S_{X,b} L_{sigma,b}^T (l_tau x l_sigma), all column-major.  L_{tau,b}[i][q] =
// L[a_off + q l_tau + i] (the k_b rows of cluster tau's coefficient block that belong to b).
// Consecutive threads take consecutive rows, so the reads of a column are contiguous.
constexpr int kCoupThreads = 256;
__global__ __launch_bounds__(kCoupThreads) void k_couplings(const double2* __restrict__ L, int64_t L_len,
                                                            const double* __restrict__ sig, int64_t sig_len,
                                                            const uhm_coupling_desc* __restrict__ desc,
                                                            int64_t nblocks, double2* __restrict__ S, int64_t S_len,
                                                            double2* __restrict__ SX, int64_t SX_len,
                                                            double2* __restrict__ SY, int64_t SY_len,
                                                            int32_t* __restrict__ status) {
  const int64_t b = blockIdx.x;
  if (b >= nblocks) return;
  const uhm_coupling_desc d = desc[b];
  const int64_t lt = d.lt, ls = d.ls, kb = d.kb;
  const bool ok = lt >= 1 && ls >= 1 && kb >= 1 && d.a_off >= 0 && d.a_off + kb * lt <= L_len && d.b_off >= 0 &&
                  d.b_off + kb * ls <= L_len && d.sig_off >= 0 && d.sig_off + kb <= sig_len && d.s_off >= 0 &&
                  d.s_off + lt * ls <= S_len && d.x_off >= 0 && d.x_off + lt * kb <= SX_len && d.y_off >= 0 &&
                  d.y_off + ls * kb <= SY_len;
  if (threadIdx.x == 0) status[b] = ok ? 1 : -1;
  if (!ok) return;
  const double2* A = L + d.a_off;
  const double2* B = L + d.b_off;
  const double* sg = sig + d.sig_off;
  for (int64_t e = threadIdx.x; e < lt * kb; e += kCoupThreads) {
    const int64_t q = e / lt;
    const double inv = 1.0 / sg[q];
    const double2 a = A[e];
    SX[d.x_off + e] = make_double2(a.x * inv, a.y * inv);
  }
  for (int64_t e = threadIdx.x; e < ls * kb; e += kCoupThreads) SY[d.y_off + e] = cconj(B[e]);
  for (int64_t e = threadIdx.x; e < lt * ls; e += kCoupThreads) {
    const int64_t i = e % lt, j = e / lt;
    double ar = 0.0, ai = 0.0;
    for (int64_t q = 0; q < kb; ++q) {
      const double2 x = A[q * lt + i], y = B[q * ls + j];
      const double inv = 1.0 / sg[q];
      ar += (x.x * y.x - x.y * y.y) * inv;
      ai += (x.x * y.y + x.y * y.x) * inv;
    }
    S[d.s_off + e] = make_double2(ar, ai);
  }
}

// Row-major rows x cols matrices (the caller's layout) into column-major copies in the
// workspace, through 32 x 32 LDS tiles so that reads and writes are both contiguous.  Grid
// (ceil(cols / 32), ceil(rows / 32), batch), 256 threads.
__global__ __launch_bounds__(256) void k_to_colmajor(const double2* __restrict__ src, int64_t s_stride, int32_t rows,
                                                     int32_t cols, CArr dst) {
  __shared__ double2 tile[32][33];
  const int c = blockIdx.z;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const double2* S = src + (int64_t)c * s_stride;
  double2* D = dst.at(c);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 8 rows of 32 per pass
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, q = c0 + tx;
    tile[k][tx] = (r < rows && q < cols) ? S[(int64_t)r * cols + q] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int q = c0 + k, r = r0 + tx;
    if (q < cols && r < rows) D[(int64_t)q * rows + r] = tile[tx][k];
  }
}

// dst = src^* on the leading k x k block of two P x P column-major matrices (ld P), through
// 32 x 32 LDS tiles.  Grid (ceil(k / 32), ceil(k / 32), batch), 256 threads.
__global__ __launch_bounds__(256) void k_ctrans(CArr src, CArr dst, int32_t P, int32_t k) {
  __shared__ double2 tile[32][33];
  const int c = blockIdx.z;
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;  // a tile of src: rows r0.., columns c0..
  const double2* S = src.at(c);
  double2* D = dst.at(c);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int q = ty; q < 32; q += 8) {  // column c0 + q of src, rows r0 + tx
    const int r = r0 + tx, col = c0 + q;
    tile[q][tx] = (r < k && col < k) ? S[(int64_t)col * P + r] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {  // column r0 + q of dst, rows c0 + tx: src(r0 + q, c0 + tx)^*
    const int r = c0 + tx, col = r0 + q;
    if (r < k && col < k) {
      const double2 v = tile[tx][q];
      D[(int64_t)col * P + r] = make_double2(v.x, -v.y);
    }
  }
}

int to_colmajor(const double* src, int32_t batch, int32_t rows, int32_t cols, CArr dst, hipStream_t s) {
  k_to_colmajor<<<dim3((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32), (unsigned)batch), dim3(256), 0, s>>>(
      reinterpret_cast<const double2*>(src), (int64_t)rows * cols, rows, cols, dst);
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

// Per-matrix workspace of the cluster factorisation (offsets in doubles).
struct ClusterWs {
  int64_t per, o_x, o_w, o_om, o_c, o_cq, o_r2, o_j, o_nu, o_ord, o_st;
};
ClusterWs cluster_ws(int32_t m, int32_t n, int32_t P) {
  Carve cv;
  ClusterWs w{};
  w.o_x = cv.take(2 * (int64_t)m * n);  // the column-major copy of X, factorised in place
  w.o_w = cv.take(2 * (int64_t)P * m);
  w.o_om = cv.take(P);
  w.o_c = cv.take(2 * (int64_t)n * P);
  w.o_cq = cv.take(2 * (int64_t)n * P);
  w.o_r2 = cv.take(2 * (int64_t)P * P);
  w.o_j = cv.take(2 * (int64_t)P * P);
  w.o_nu = cv.take(2 * (int64_t)std::max(n, P));
  w.o_ord = cv.take((P + 1) / 2);
  // ints [0..3] the pivoted QR, [4..7] the QR of B^*, [8..11] Jacobi; doubles from 8:
  // ||X||_F^2, T^2
  w.o_st = cv.take(32);
  w.per = cv.per;
  return w;
}

// Per-matrix workspace of the recompression (offsets in doubles).
struct RecWs {
  int64_t per, o_x, o_y, o_wx, o_omx, o_wy, o_omy, o_rx, o_ry, o_m, o_j, o_qj, o_qw, o_nux, o_nuy, o_ord, o_st;
};
RecWs rec_ws(int32_t m, int32_t n, int32_t kp) {
  Carve cv;
  RecWs w{};
  const int64_t kk = 2 * (int64_t)kp * kp;
  w.o_x = cv.take(2 * (int64_t)m * kp);  // column-major copies of the factors
  w.o_y = cv.take(2 * (int64_t)n * kp);
  w.o_wx = cv.take(2 * (int64_t)kp * m);
  w.o_omx = cv.take(kp);
  w.o_wy = cv.take(2 * (int64_t)kp * n);
  w.o_omy = cv.take(kp);
  w.o_rx = cv.take(kk);
  w.o_ry = cv.take(kk);
  w.o_m = cv.take(kk);
  w.o_j = cv.take(kk);
  w.o_qj = cv.take(kk);
  w.o_qw = cv.take(kk);
  w.o_nux = cv.take(2 * (int64_t)kp);
  w.o_nuy = cv.take(2 * (int64_t)kp);
  w.o_ord = cv.take((kp + 1) / 2);
  w.o_st = cv.take(32);  // ints [0..3] the QR of X, [4..7] the QR of Y, [8..11] Jacobi
  w.per = cv.per;
  return w;
}

// The steps of one QR over a batch: a wavefront per column up to 512 rows, else a
// workgroup of 128 to 1024 threads per column (8 rows per thread; 16 above 8192 rows).
int run_qr(const QrStep& q, int32_t batch, int32_t steps, hipStream_t s) {
  if (q.rows > 16 * kBigThreads) return fail(UHM_EINVAL, "QR step: more than 16384 rows");
  const dim3 gn((unsigned)((q.cols + kStepCols - 1) / kStepCols), (unsigned)batch);
  const dim3 gw((unsigned)((q.cols + kWideCols - 1) / kWideCols), (unsigned)batch);
  for (int32_t k = 0; k <= steps; ++k) {
    if (q.rows <= 64 * 8)
      k_qr_step<8><<<gn, dim3(kStepThreads), 0, s>>>(q, k);
    else if (q.rows <= 128 * 8)
      k_qr_step_wide<128, 8><<<gw, dim3(128), 0, s>>>(q, k);
    else if (q.rows <= 256 * 8)
      k_qr_step_wide<256, 8><<<gw, dim3(256), 0, s>>>(q, k);
    else if (q.rows <= 512 * 8)
      k_qr_step_wide<512, 8><<<gw, dim3(512), 0, s>>>(q, k);
    else if (q.rows <= 1024 * 8)
      k_qr_step_wide<1024, 8><<<gw, dim3(1024), 0, s>>>(q, k);
    else
      k_qr_step_wide<1024, 16><<<gw, dim3(1024), 0, s>>>(q, k);
    UHM_HIP(hipGetLastError());
  }
  return UHM_OK;
}

double jacobi_tol(int32_t P) { return std::sqrt((double)P) * 2.220446049250313e-16; }

}  // namespace
}  // namespace uhm_detail

using namespace uhm_detail;

extern "C" {

int64_t uhm_cluster_basis_work(int32_t batch, int32_t m, int32_t n, int32_t pmax) {
  if (batch < 0 || m < 1 || n < 1 || pmax < 1) return -1;
  return cluster_ws(m, n, pmax).per * (int64_t)batch + 32;
}

int uhm_cluster_basis(const double* X, int32_t batch, int32_t m, int32_t n, int32_t pmax, double tol, double eps,
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
  const int32_t P = pmax;
  const ClusterWs ws = cluster_ws(m, n, P);
  if (work_len < ws.per * (int64_t)batch + 32) return fail(UHM_EINVAL, "uhm_cluster_basis: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  UHM_HIP(hipMemsetAsync(work, 0, sizeof(double) * (size_t)(ws.per * (int64_t)batch), s));
  const int64_t per = ws.per;
  const CArr Xa = region<double2>(work, per, ws.o_x);
  int rc;
  if ((rc = to_colmajor(X, batch, m, n, Xa, s))) return rc;
  const CArr Wa = region<double2>(work, per, ws.o_w), Ca = region<double2>(work, per, ws.o_c),
             Cq = region<double2>(work, per, ws.o_cq), R2 = region<double2>(work, per, ws.o_r2),
             Ja = region<double2>(work, per, ws.o_j);
  const DArr om = region<double>(work, per, ws.o_om), nu = region<double>(work, per, ws.o_nu),
             fro = region<double>(work, per, ws.o_st + 8);
  const IArr ord = region<int32_t>(work, per, ws.o_ord), st = region<int32_t>(work, per, ws.o_st);
  const IArr stA = st, stB{st.p + 4, st.stride}, stS{st.p + 8, st.stride};
  const CArr none{nullptr, 0};
  const DArr dnone{nullptr, 0};
  const IArr inone{nullptr, 0};
  const int32_t kcap = std::min(std::min(m, n), P);

  // 1. pivoted QR of X to the tolerance; B^* into C (kept) and Cq (consumed by step 2)
  k_col_norms<<<dim3((unsigned)((n + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(
      Xa, m, n, nu);
  UHM_HIP(hipGetLastError());
  const QrStep q1{Xa, m, n, nu, Wa, om, Ca, Cq, n, 1, 1, stA, inone, fro, kcap, tol * tol, 1};
  if ((rc = run_qr(q1, batch, kcap, s))) return rc;
  // the batch's largest p sizes the steps of the QR of B^* and the Jacobi schedule
  int32_t* dmax = reinterpret_cast<int32_t*>(work + ws.per * (int64_t)batch) + 1;
  UHM_HIP(hipMemsetAsync(dmax, 0, sizeof(int32_t), s));
  k_batch_max<<<dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s>>>(stA, batch, dmax);
  UHM_HIP(hipGetLastError());
  int32_t pbat = 0;
  UHM_HIP(hipMemcpyAsync(&pbat, dmax, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  UHM_HIP(hipStreamSynchronize(s));
  if (pbat < 0 || pbat > P) return fail(UHM_EHIP, "uhm_cluster_basis: QR step count out of range");
  // 2. QR of B^* (n x pbat: the columns beyond are zero in every matrix; column-major in Cq):
  // R2 (ld P)
  const int32_t pc = std::max(pbat, 1);
  k_col_norms<<<dim3((unsigned)((pc + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(
      Cq, n, pc, nu);
  UHM_HIP(hipGetLastError());
  const QrStep q2{Cq, n, pc, nu, none, dnone, R2, none, 1, P, 0, stB, stA, dnone, P, 0.0, 0};
  if ((rc = run_qr(q2, batch, pbat, s))) return rc;
  // 3. one-sided Jacobi on the columns of M = R2^* (in Ja; B = R2^* Q2^*, so the left
  // singular vectors of B are those of M): M J = W Sigma, and W's columns are the rotated
  // columns scaled by 1 / sigma, so the rotations J need not be kept.  Then the rank rule,
  // and the kept columns of M J orthonormalised (into R2).
  if (pbat > 0) {
    const unsigned tk = (unsigned)((pbat + 31) / 32);
    k_ctrans<<<dim3(tk, tk, (unsigned)batch), dim3(256), 0, s>>>(R2, Ja, P, pbat);
    UHM_HIP(hipGetLastError());
  }
  if ((rc = run_jacobi(Ja, none, P, pbat, stA, stS, batch, jacobi_tol(P), 60,
                       reinterpret_cast<int32_t*>(work + ws.per * (int64_t)batch), s)))
    return rc;
  const Finish f{Ja, P, stA, stS, ord, eps, fro, stA, m, n, sv, rank, psteps, stats, status};
  k_finish<<<dim3((unsigned)batch), dim3(kStepThreads), 0, s>>>(f);
  UHM_HIP(hipGetLastError());
  k_orth<<<dim3((unsigned)batch), dim3(kBigThreads), 0, s>>>(Ja, P, ord, stA, stS, R2, P);
  UHM_HIP(hipGetLastError());
  // 4. U = Q_p [Jo; 0] and Sigma V^* = Jo^* B
  const Apply ap{Wa, om, m, stA, R2, P, stA, stS, CArr{reinterpret_cast<double2*>(U), (int64_t)m * P}};
  if ((rc = launch_apply(ap, P, batch, s))) return rc;
  k_fac_sv<<<dim3((unsigned)((n + kSvT - 1) / kSvT), (unsigned)((P + kSvT - 1) / kSvT), (unsigned)batch),
             dim3(kSvT * kSvT), 0, s>>>(R2, P, stA, stS, Ca, n, reinterpret_cast<double2*>(SV));
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

int64_t uhm_block_recompress_work(int32_t batch, int32_t m, int32_t n, int32_t kp) {
  if (batch < 0 || m < 1 || n < 1 || kp < 1) return -1;
  return rec_ws(m, n, kp).per * (int64_t)batch + 32;
}

int uhm_block_recompress(const double* X, const double* Y, int32_t batch, int32_t m, int32_t n, int32_t kp, double eps,
                         double* U, double* V, double* sv, int32_t* rank, int32_t* status, double* work,
                         int64_t work_len, void* hip_stream) {
  if (batch < 0 || m < 1 || n < 1) return fail(UHM_EINVAL, "uhm_block_recompress: bad size");
  if (m > kFacMaxRows || n > kFacMaxRows) return fail(UHM_EINVAL, "uhm_block_recompress: more than 16384 rows");
  if (kp < 1 || kp > kFacMaxP || kp > std::min(m, n))
    return fail(UHM_EINVAL, "uhm_block_recompress: kp must be in 1..min(m, n, 2048)");
  if (!(eps >= 0.0) || !std::isfinite(eps))
    return fail(UHM_EINVAL, "uhm_block_recompress: eps must be finite and >= 0");
  if (batch == 0) return UHM_OK;
  if (batch > 65535) return fail(UHM_EINVAL, "uhm_block_recompress: more than 65535 blocks in one call");
  if (!X || !Y || !U || !V || !sv || !rank || !status || !work)
    return fail(UHM_EINVAL, "uhm_block_recompress: null pointer");
  const RecWs ws = rec_ws(m, n, kp);
  if (work_len < ws.per * (int64_t)batch + 32)
    return fail(UHM_EINVAL, "uhm_block_recompress: workspace too small");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  UHM_HIP(hipMemsetAsync(work, 0, sizeof(double) * (size_t)(ws.per * (int64_t)batch), s));
  const int64_t per = ws.per;
  const CArr Xa = region<double2>(work, per, ws.o_x), Ya = region<double2>(work, per, ws.o_y);
  int rc;
  if ((rc = to_colmajor(X, batch, m, kp, Xa, s)) || (rc = to_colmajor(Y, batch, n, kp, Ya, s))) return rc;
  const CArr WX = region<double2>(work, per, ws.o_wx), WY = region<double2>(work, per, ws.o_wy),
             RX = region<double2>(work, per, ws.o_rx), RY = region<double2>(work, per, ws.o_ry),
             Ma = region<double2>(work, per, ws.o_m), Ja = region<double2>(work, per, ws.o_j),
             QJ = region<double2>(work, per, ws.o_qj), QW = region<double2>(work, per, ws.o_qw);
  const DArr omx = region<double>(work, per, ws.o_omx), omy = region<double>(work, per, ws.o_omy),
             nux = region<double>(work, per, ws.o_nux), nuy = region<double>(work, per, ws.o_nuy);
  const IArr ord = region<int32_t>(work, per, ws.o_ord), st = region<int32_t>(work, per, ws.o_st);
  const IArr stX = st, stY{st.p + 4, st.stride}, stS{st.p + 8, st.stride};
  const CArr none{nullptr, 0};
  const DArr dnone{nullptr, 0};
  const IArr inone{nullptr, 0};
  // 1. unpivoted QR of both factors (all kp steps), R upper triangular (ld kp)
  k_col_norms<<<dim3((unsigned)((kp + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(
      Xa, m, kp, nux);
  UHM_HIP(hipGetLastError());
  k_col_norms<<<dim3((unsigned)((kp + kStepCols - 1) / kStepCols), (unsigned)batch), dim3(kStepThreads), 0, s>>>(
      Ya, n, kp, nuy);
  UHM_HIP(hipGetLastError());
  const QrStep qx{Xa, m, kp, nux, WX, omx, RX, none, 1, kp, 0, stX, inone, dnone, kp, 0.0, 0};
  const QrStep qy{Ya, n, kp, nuy, WY, omy, RY, none, 1, kp, 0, stY, inone, dnone, kp, 0.0, 0};
  if ((rc = run_qr(qx, batch, kp, s))) return rc;
  if ((rc = run_qr(qy, batch, kp, s))) return rc;
  // 2. M = R_Y R_X^*; one-sided Jacobi M J = W Sigma (order kp = the steps of the QR of X)
  k_rr<<<dim3((unsigned)((kp + 15) / 16), (unsigned)((kp + 15) / 16), (unsigned)batch), dim3(256), 0, s>>>(RY, RX, kp,
                                                                                                         Ma);
  UHM_HIP(hipGetLastError());
  if ((rc = run_jacobi(Ma, Ja, kp, kp, stX, stS, batch, jacobi_tol(kp), 60,
                       reinterpret_cast<int32_t*>(work + ws.per * (int64_t)batch), s)))
    return rc;
  const Finish f{Ma, kp, stX, stS, ord, eps, dnone, inone, m, n, sv, rank, nullptr, nullptr, status};
  k_finish<<<dim3((unsigned)batch), dim3(kStepThreads), 0, s>>>(f);
  UHM_HIP(hipGetLastError());
  // 3. the kept columns of J and of M J (normalised) orthonormalised, then U = Q_X [J_k; 0]
  // and V = Q_Y [W_k; 0]
  k_orth<<<dim3((unsigned)batch), dim3(kBigThreads), 0, s>>>(Ja, kp, ord, stX, stS, QJ, kp);
  UHM_HIP(hipGetLastError());
  k_orth<<<dim3((unsigned)batch), dim3(kBigThreads), 0, s>>>(Ma, kp, ord, stX, stS, QW, kp);
  UHM_HIP(hipGetLastError());
  const Apply au{WX, omx, m, stX, QJ, kp, stX, stS, CArr{reinterpret_cast<double2*>(U), (int64_t)m * kp}};
  if ((rc = launch_apply(au, kp, batch, s))) return rc;
  const Apply av{WY, omy, n, stY, QW, kp, stX, stS, CArr{reinterpret_cast<double2*>(V), (int64_t)n * kp}};
  if ((rc = launch_apply(av, kp, batch, s))) return rc;
  return UHM_OK;
}

int uhm_couplings(const double* L, int64_t L_len, const double* sigma, int64_t sigma_len,
                  const uhm_coupling_desc* blocks, int64_t nblocks, double* S, int64_t S_len, double* SX, int64_t SX_len,
                  double* SY, int64_t SY_len, int32_t* status, void* hip_stream) {
  if (L_len < 0 || sigma_len < 0 || nblocks < 0 || S_len < 0 || SX_len < 0 || SY_len < 0)
    return fail(UHM_EINVAL, "uhm_couplings: negative size");
  if (nblocks == 0) return UHM_OK;
  if (!L || !sigma || !blocks || !S || !SX || !SY || !status) return fail(UHM_EINVAL, "uhm_couplings: null pointer");
  if (nblocks > INT32_MAX) return fail(UHM_EINVAL, "uhm_couplings: too many blocks for one launch");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  k_couplings<<<dim3((unsigned)nblocks), dim3(kCoupThreads), 0, s>>>(
      reinterpret_cast<const double2*>(L), L_len, sigma, sigma_len, blocks, nblocks, reinterpret_cast<double2*>(S),
      S_len, reinterpret_cast<double2*>(SX), SX_len, reinterpret_cast<double2*>(SY), SY_len, status);
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

}  // extern "C"
