// Construction on the GPU: blocks of the kernel matrix and ACA with partial pivoting.
//
// In the paper's setting, sampling matrix entries dominates the construction (section 4.3:
// the entry cost C_elem multiplies every term of the construction count), and ACA (section
// 2.3) samples k rows and k columns of each admissible block.  Here every entry is the
// Helmholtz single-layer kernel at a point pair (section 6.1), evaluated where it is used.
//
// k_kernel_blocks: one workgroup per dense block; consecutive lanes write consecutive
// entries of a column (coalesced column-major stores).
//
// k_aca: one workgroup of W wavefronts per block, W = 1..16 chosen per launch from the
// largest block (about 8 rows per thread).  Thread t owns rows t, t+64W, ... and columns
// t, t+64W, ... of its block: it evaluates those entries, keeps their residual updates,
// writes them into u_k and v_k, and later reads back only what it wrote itself.  The only
// values that cross threads go through LDS or reductions: the pivot row's entries u_l[i_k]
// and the pivot column's entries v_l[j_k] (gathered by their owning thread into LDS), the
// used-row flags (a bitmask in LDS), and the argmax and norm reductions (xor butterflies
// within a wavefront, then the W wavefront results combined in order, so every thread
// holds bit-identical results and takes the same branch).  Entries and factors do not
// depend on W; only the summation order of the norms in the stopping test does.
#include "uhm_internal.h"

#include <climits>
#include <cmath>

namespace uhm_detail {
namespace {

constexpr double kFourPi = 12.566370614359172953850573533118;
constexpr int kAcaMaxRows = 65536;
constexpr int kAcaMaxCap = 1024;
constexpr int kDenseThreads = 256;

__device__ __forceinline__ double2 kernel_entry(const double* __restrict__ p, const double* __restrict__ q,
                                                bool same, double kappa, double diag) {
  const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  if (same || r == 0.0) return make_double2(diag, 0.0);
  const double s = 1.0 / (kFourPi * r);
  double sn, cs;
  sincos(kappa * r, &sn, &cs);
  return make_double2(cs * s, sn * s);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

struct Pick {
  double mag;  // re^2 + im^2
  int idx;
  double re, im;
};

// Largest modulus, smallest index on ties: a total order, so every lane ends with the same pick.
__device__ __forceinline__ Pick wave_argmax(Pick a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Pick b;
    b.mag = __shfl_xor(a.mag, o, 64);
    b.idx = __shfl_xor(a.idx, o, 64);
    b.re = __shfl_xor(a.re, o, 64);
    b.im = __shfl_xor(a.im, o, 64);
    if (b.mag > a.mag || (b.mag == a.mag && b.idx < a.idx)) a = b;
  }
  return a;
}

__global__ __launch_bounds__(kDenseThreads) void k_kernel_blocks(
    const double* __restrict__ pts, int64_t npts, double kappa, double diag, const uhm_block_desc* __restrict__ blocks,
    double2* __restrict__ D, int64_t D_len, int32_t* __restrict__ status) {
  const int64_t b = blockIdx.x;
  const uhm_block_desc B = blocks[b];
  const int64_t m = B.rows, n = B.cols;
  const bool ok = m >= 1 && n >= 1 && B.row_off >= 0 && B.col_off >= 0 && B.row_off + m <= npts &&
                  B.col_off + n <= npts && B.a_off >= 0 && B.a_off + m * n <= D_len;
  if (threadIdx.x == 0) status[b] = ok ? 1 : -1;
  if (!ok) return;
  const double* P = pts + 3 * B.row_off;
  const double* Q = pts + 3 * B.col_off;
  double2* out = D + B.a_off;
  const int64_t shift = B.col_off - B.row_off;  // row i and column j are one point when i == j + shift
  for (int64_t e = threadIdx.x; e < m * n; e += kDenseThreads) {
    const int64_t j = e / m, i = e - j * m;
    out[e] = kernel_entry(P + 3 * i, Q + 3 * j, i == j + shift, kappa, diag);
  }
}

// Combines one value per wavefront, in wavefront order, so that every thread of the block
// holds the same result.  `slot` has W entries; a barrier separates the writes from the reads.
template <int W>
__device__ __forceinline__ double block_sum(double x, double* slot) {
  x = wave_sum(x);
  if (W == 1) return x;
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = x;
  __syncthreads();
  double s = 0.0;
#pragma unroll 1
  for (int w = 0; w < W; ++w) s += slot[w];
  return s;
}

template <int W>
__device__ __forceinline__ Pick block_argmax(Pick a, Pick* slot) {
  a = wave_argmax(a);
  if (W == 1) return a;
  if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = a;
  __syncthreads();
  Pick r = slot[0];
#pragma unroll 1
  for (int w = 1; w < W; ++w) {
    const Pick b = slot[w];
    if (b.mag > r.mag || (b.mag == r.mag && b.idx < r.idx)) r = b;
  }
  return r;
}

constexpr int kCrossGroup = 4;  // norm cross terms reduced 4 at a time

// W wavefronts per block (64 W threads).  Thread t owns rows t, t + 64W, ... and columns
// t, t + 64W, ... of its block; every value it reads back from U or V it wrote itself.
// Everything that decides a branch (pivots, norms, the stopping test) is combined in a fixed
// order and is bit-identical in all threads, so all threads take every branch together.
template <int W>
__global__ __launch_bounds__(64 * W) void k_aca(const double* __restrict__ pts, int64_t npts, double kappa,
                                                double diag, const uhm_block_desc* __restrict__ blocks,
                                                int32_t max_rows, int32_t max_cap, double eps, double2* U,
                                                int64_t U_len, double2* V, int64_t V_len, int32_t* piv,
                                                int64_t piv_len, int32_t* __restrict__ rank_out,
                                                int32_t* __restrict__ status_out) {
  constexpr int T = 64 * W;
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ Pick red_row[W], red_col[W];
  __shared__ double red_nv[W], red_nu[W];
  __shared__ int red_free[W];
  __shared__ double red_cross[2][W][4 * kCrossGroup];
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x;
  const uhm_block_desc B = blocks[b];
  const int m = B.rows, n = B.cols, cap = B.cap;
  const bool ok = m >= 1 && n >= 1 && cap >= 1 && m <= max_rows && cap <= max_cap && B.row_off >= 0 &&
                  B.col_off >= 0 && B.row_off + m <= npts && B.col_off + n <= npts && B.a_off >= 0 &&
                  B.a_off + (int64_t)m * cap <= U_len && B.b_off >= 0 && B.b_off + (int64_t)n * cap <= V_len &&
                  B.p_off >= 0 && B.p_off + 2 * (int64_t)cap <= piv_len;
  if (!ok) {
    if (tid == 0) {
      rank_out[b] = 0;
      status_out[b] = -1;
    }
    return;
  }
  double2* ui = reinterpret_cast<double2*>(lds);  // u_l[i_k], l < k
  double2* vj = ui + max_cap;                     // v_l[j_k], l < k
  uint32_t* used = reinterpret_cast<uint32_t*>(vj + max_cap);
  const int nwords = (m + 31) >> 5;
  for (int w = tid; w < nwords; w += T) used[w] = 0u;

  double2* u = U + B.a_off;
  double2* v = V + B.b_off;
  int32_t* prow = piv + B.p_off;
  int32_t* pcol = prow + cap;
  const double* P = pts + 3 * B.row_off;
  const double* Q = pts + 3 * B.col_off;
  const int64_t shift = B.col_off - B.row_off;
  const int kmax = min(min(m, n), cap);
  int k = 0, i = 0, status = -2;  // -2: the term limit ended the loop
  double norm2 = 0.0;             // |S_k|_F^2
  __syncthreads();

  while (k < kmax) {
    // u_l[i] for l < k, gathered by the thread that wrote row i
    if (tid == i % T)
      for (int l = 0; l < k; ++l) ui[l] = u[(size_t)l * m + i];
    __syncthreads();
    // residual row i (unscaled) into v column k, and its largest entry
    const double* pi = P + 3 * (int64_t)i;
    double2* vk = v + (size_t)k * n;
    Pick best{-1.0, INT_MAX, 0.0, 0.0};
    for (int j = tid; j < n; j += T) {
      double2 a = kernel_entry(pi, Q + 3 * (int64_t)j, (int64_t)i == (int64_t)j + shift, kappa, diag);
      for (int l = 0; l < k; ++l) {
        const double2 w = ui[l];
        const double2 z = v[(size_t)l * n + j];
        a.x -= w.x * z.x - w.y * z.y;
        a.y -= w.x * z.y + w.y * z.x;
      }
      vk[j] = a;
      const double mg = a.x * a.x + a.y * a.y;
      if (mg > best.mag) best = Pick{mg, j, a.x, a.y};
    }
    if (tid == 0) used[i >> 5] |= 1u << (i & 31);
    best = block_argmax<W>(best, red_row);
    __syncthreads();  // the used flag of row i
    if (!(best.mag > 0.0)) {
      // the residual row vanishes: retry with the unused row of smallest index
      int nx = INT_MAX;
      for (int w = tid; w < nwords; w += T) {
        const uint32_t freebits = ~used[w] & (w == nwords - 1 && (m & 31) ? ((1u << (m & 31)) - 1u) : 0xffffffffu);
        if (freebits) {
          nx = (w << 5) + __builtin_ctz(freebits);
          break;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) nx = min(nx, __shfl_xor(nx, o, 64));
      if (W > 1) {
        if ((tid & 63) == 0) red_free[tid >> 6] = nx;
        __syncthreads();
        for (int w = 0; w < W; ++w) nx = min(nx, red_free[w]);
        __syncthreads();
      }
      if (nx == INT_MAX) {
        status = 2;
        break;
      }
      i = nx;
      continue;
    }
    const int jp = best.idx;
    const double dd = best.re * best.re + best.im * best.im;
    const double ir = best.re / dd, ii = -best.im / dd;  // 1 / r[j_k]
    double nv = 0.0;
    for (int j = tid; j < n; j += T) {
      const double2 a = vk[j];
      const double2 z = make_double2(a.x * ir - a.y * ii, a.x * ii + a.y * ir);
      vk[j] = z;
      nv += z.x * z.x + z.y * z.y;
    }
    // v_l[j_k] for l < k, gathered by the thread that wrote column j_k
    if (tid == jp % T)
      for (int l = 0; l < k; ++l) vj[l] = v[(size_t)l * n + jp];
    nv = block_sum<W>(nv, red_nv);
    __syncthreads();  // vj
    // residual column j_k into u column k; |u_k|^2; next pivot among the unused rows
    const double* qj = Q + 3 * (int64_t)jp;
    double2* uk = u + (size_t)k * m;
    double nu = 0.0;
    Pick nxt{-1.0, INT_MAX, 0.0, 0.0};
    for (int t = tid; t < m; t += T) {
      double2 a = kernel_entry(P + 3 * (int64_t)t, qj, (int64_t)t == (int64_t)jp + shift, kappa, diag);
      for (int l = 0; l < k; ++l) {
        const double2 w = vj[l];
        const double2 z = u[(size_t)l * m + t];
        a.x -= w.x * z.x - w.y * z.y;
        a.y -= w.x * z.y + w.y * z.x;
      }
      uk[t] = a;
      const double mg = a.x * a.x + a.y * a.y;
      nu += mg;
      if (!((used[t >> 5] >> (t & 31)) & 1u) && mg > nxt.mag) nxt = Pick{mg, t, 0.0, 0.0};
    }
    nu = block_sum<W>(nu, red_nu);
    nxt = block_argmax<W>(nxt, red_col);
    // |S_k|^2 = |S_{k-1}|^2 + 2 Re sum_{l<k} (u_l^* u_k)(v_l^* v_k) + |u_k|^2 |v_k|^2,
    // the inner products taken kCrossGroup at a time
    double cross = 0.0;
    for (int l0 = 0, g = 0; l0 < k; l0 += kCrossGroup, ++g) {
      const int cnt = min(kCrossGroup, k - l0);
      double acc[4 * kCrossGroup];
#pragma unroll
      for (int q = 0; q < 4 * kCrossGroup; ++q) acc[q] = 0.0;
      for (int t = tid; t < m; t += T) {
        const double2 y = uk[t];
#pragma unroll
        for (int q = 0; q < kCrossGroup; ++q) {
          if (q < cnt) {
            const double2 x = u[(size_t)(l0 + q) * m + t];
            acc[4 * q] += x.x * y.x + x.y * y.y;
            acc[4 * q + 1] += x.x * y.y - x.y * y.x;
          }
        }
      }
      for (int j = tid; j < n; j += T) {
        const double2 y = vk[j];
#pragma unroll
        for (int q = 0; q < kCrossGroup; ++q) {
          if (q < cnt) {
            const double2 x = v[(size_t)(l0 + q) * n + j];
            acc[4 * q + 2] += x.x * y.x + x.y * y.y;
            acc[4 * q + 3] += x.x * y.y - x.y * y.x;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 4 * kCrossGroup; ++q) acc[q] = wave_sum(acc[q]);
      if (W > 1) {
        double* slot = red_cross[g & 1][0];
        if ((tid & 63) == 0) {
#pragma unroll
          for (int q = 0; q < 4 * kCrossGroup; ++q) slot[(tid >> 6) * 4 * kCrossGroup + q] = acc[q];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4 * kCrossGroup; ++q) {
          double s = 0.0;
#pragma unroll 1
          for (int w = 0; w < W; ++w) s += slot[w * 4 * kCrossGroup + q];
          acc[q] = s;
        }
      }
#pragma unroll
      for (int q = 0; q < kCrossGroup; ++q)
        if (q < cnt) cross += acc[4 * q] * acc[4 * q + 2] - acc[4 * q + 1] * acc[4 * q + 3];
    }
    norm2 += 2.0 * cross + nu * nv;
    if (tid == 0) {
      prow[k] = i;
      pcol[k] = jp;
    }
    ++k;
    if (sqrt(nu * nv) <= eps * sqrt(fmax(norm2, 0.0))) {
      status = 1;
      break;
    }
    if (nxt.idx == INT_MAX) {
      status = 2;
      break;
    }
    i = nxt.idx;
  }
  if (status == -2) status = (kmax == min(m, n)) ? 2 : 0;
  if (tid == 0) {
    rank_out[b] = k;
    status_out[b] = status;
  }
}

// Packing of ACA factors for the recompression: one workgroup per selected block, one
// thread per packed element in output order (row-major m x kp, then n x kp), so the writes
// are contiguous; the reads walk the column-major factors, whose lines the workgroup's
// neighbouring rows reuse from the caches.
constexpr int kPackThreads = 256;
__global__ __launch_bounds__(kPackThreads) void k_aca_pack(const uhm_block_desc* __restrict__ blocks, int64_t nblocks,
                                                           const int32_t* __restrict__ rank,
                                                           const double2* __restrict__ U, int64_t U_len,
                                                           const double2* __restrict__ V, int64_t V_len,
                                                           const int32_t* __restrict__ sel, int32_t m, int32_t n,
                                                           int32_t kp, double2* __restrict__ X, double2* __restrict__ Y,
                                                           int32_t* __restrict__ status) {
  const int c = blockIdx.x;
  const int32_t b = sel[c];
  bool ok = b >= 0 && b < nblocks;
  uhm_block_desc d{};
  int32_t k = 0;
  if (ok) {
    d = blocks[b];
    k = rank[b];
    ok = d.rows == m && d.cols == n && k >= 0 && k <= kp && k <= d.cap && d.a_off >= 0 && d.b_off >= 0 &&
         d.a_off + (int64_t)k * m <= U_len && d.b_off + (int64_t)k * n <= V_len;
  }
  if (!ok) k = 0;  // a rejected block is written as zeros
  double2* Xc = X + (int64_t)c * m * kp;
  double2* Yc = Y + (int64_t)c * n * kp;
  for (int64_t q = threadIdx.x; q < (int64_t)m * kp; q += kPackThreads) {
    const int i = (int)(q / kp), l = (int)(q - (int64_t)i * kp);
    Xc[q] = l < k ? U[d.a_off + (int64_t)l * m + i] : make_double2(0.0, 0.0);
  }
  for (int64_t q = threadIdx.x; q < (int64_t)n * kp; q += kPackThreads) {
    const int j = (int)(q / kp), l = (int)(q - (int64_t)j * kp);
    const double2 v = l < k ? V[d.b_off + (int64_t)l * n + j] : make_double2(0.0, 0.0);
    Yc[q] = make_double2(v.x, -v.y);
  }
  if (threadIdx.x == 0) status[c] = ok ? 1 : -1;
}

// Wavefronts per block for a launch: enough that each thread holds about 8 of the largest
// block's rows, between 1 and 16.
int aca_waves(int32_t max_rows) {
  int w = 1;
  while (w < 16 && 512 * w < max_rows) w *= 2;
  return w;
}

}  // namespace
}  // namespace uhm_detail

using namespace uhm_detail;

extern "C" {

int uhm_kernel_blocks(const double* points, int64_t npoints, double kappa, double diag, const uhm_block_desc* blocks,
                      int64_t nblocks, double* D, int64_t D_len, int32_t* status, void* hip_stream) {
  if (npoints < 0 || nblocks < 0 || D_len < 0) return fail(UHM_EINVAL, "uhm_kernel_blocks: negative size");
  if (nblocks == 0) return UHM_OK;
  if (!points || !blocks || !D || !status) return fail(UHM_EINVAL, "uhm_kernel_blocks: null pointer");
  if (nblocks > INT32_MAX) return fail(UHM_EINVAL, "uhm_kernel_blocks: too many blocks for one launch");
  if (!std::isfinite(kappa) || !std::isfinite(diag)) return fail(UHM_EINVAL, "uhm_kernel_blocks: kappa/diag not finite");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  k_kernel_blocks<<<dim3((unsigned)nblocks), dim3(kDenseThreads), 0, s>>>(
      points, npoints, kappa, diag, blocks, reinterpret_cast<double2*>(D), D_len, status);
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

int uhm_aca(const double* points, int64_t npoints, double kappa, double diag, const uhm_block_desc* blocks,
            int64_t nblocks, int32_t max_rows, int32_t max_cap, double eps, double* U, int64_t U_len, double* V,
            int64_t V_len, int32_t* piv, int64_t piv_len, int32_t* rank, int32_t* status, void* hip_stream) {
  if (npoints < 0 || nblocks < 0 || U_len < 0 || V_len < 0 || piv_len < 0)
    return fail(UHM_EINVAL, "uhm_aca: negative size");
  if (max_rows < 1 || max_rows > kAcaMaxRows) return fail(UHM_EINVAL, "uhm_aca: max_rows must be in 1..65536");
  if (max_cap < 1 || max_cap > kAcaMaxCap) return fail(UHM_EINVAL, "uhm_aca: max_cap must be in 1..1024");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(UHM_EINVAL, "uhm_aca: eps must be finite and >= 0");
  if (!std::isfinite(kappa) || !std::isfinite(diag)) return fail(UHM_EINVAL, "uhm_aca: kappa/diag not finite");
  if (nblocks == 0) return UHM_OK;
  if (!points || !blocks || !U || !V || !piv || !rank || !status) return fail(UHM_EINVAL, "uhm_aca: null pointer");
  if (nblocks > INT32_MAX) return fail(UHM_EINVAL, "uhm_aca: too many blocks for one launch");
  const size_t lds = 2 * sizeof(double2) * (size_t)max_cap + 4 * (size_t)((max_rows + 31) / 32);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const dim3 grid((unsigned)nblocks);
  double2* Uc = reinterpret_cast<double2*>(U);
  double2* Vc = reinterpret_cast<double2*>(V);
  switch (aca_waves(max_rows)) {
#define UHM_ACA_LAUNCH(WV)                                                                                     \
  case WV:                                                                                                     \
    k_aca<WV><<<grid, dim3(64 * WV), lds, s>>>(points, npoints, kappa, diag, blocks, max_rows, max_cap, eps, Uc, \
                                               U_len, Vc, V_len, piv, piv_len, rank, status);                 \
    break;
    UHM_ACA_LAUNCH(1)
    UHM_ACA_LAUNCH(2)
    UHM_ACA_LAUNCH(4)
    UHM_ACA_LAUNCH(8)
    UHM_ACA_LAUNCH(16)
#undef UHM_ACA_LAUNCH
    default:
      return fail(UHM_EINVAL, "uhm_aca: internal wave count");
  }
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

int uhm_aca_pack(const uhm_block_desc* blocks, int64_t nblocks, const int32_t* rank, const double* U, int64_t U_len,
                 const double* V, int64_t V_len, const int32_t* sel, int32_t cnt, int32_t m, int32_t n, int32_t kp,
                 double* X, double* Y, int32_t* status, void* hip_stream) {
  if (nblocks < 0 || U_len < 0 || V_len < 0 || cnt < 0 || m < 1 || n < 1 || kp < 1)
    return fail(UHM_EINVAL, "uhm_aca_pack: bad size");
  if (cnt == 0) return UHM_OK;
  if (!blocks || !rank || !U || !V || !sel || !X || !Y || !status) return fail(UHM_EINVAL, "uhm_aca_pack: null pointer");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  k_aca_pack<<<dim3((unsigned)cnt), dim3(kPackThreads), 0, s>>>(
      blocks, nblocks, rank, reinterpret_cast<const double2*>(U), U_len, reinterpret_cast<const double2*>(V), V_len, sel,
      m, n, kp, reinterpret_cast<double2*>(X), reinterpret_cast<double2*>(Y), status);
  UHM_HIP(hipGetLastError());
  return UHM_OK;
}

}  // extern "C"
