// Uniform H-matrix (and H-matrix) matrix-vector products for gfx950 (MI355X).
//
// Device layout (built by uhm_upload from the host image of include/uhm.h):
//
//  Forward panel F_lambda, one per leaf lambda: the rows of lambda of every basis V_sigma
//    of an ancestor sigma (root first), side by side: F_lambda = [V_s1|lambda, V_s2|lambda, ...]
//    (n_lambda x C_lambda).  It is stored tile-major: 64-column tiles, each tile row-major,
//    so one wavefront streams one contiguous tile with one lane per column and needs no
//    cross-lane reduction: lane c accumulates conj(F[i,c]) x_i over the leaf rows i.
//    The per-leaf partial sums are added over the leaves of each cluster in a fixed order
//    (deterministic), giving u_sigma = V_sigma^* v|_sigma (Algorithm 6, first loop).
//  Couplings: the blocks of row cluster tau, [S_b1 S_b2 ...] (l_tau x K_tau), are stored in
//    row chunks of at most 64 rows, each chunk column-major and contiguous.  A wavefront
//    takes a range of columns of one chunk with one lane per row (no cross-lane reduction),
//    the partial row sums go to a buffer and are added per chunk in a fixed order, giving
//    u_tau = sum_{sigma in row(tau)} S_b u_sigma (Algorithm 6, second loop).
//  Backward panel B_lambda, one per leaf: [U_t1|lambda, U_t2|lambda, ..., A|_b1, A|_b2, ...]
//    (n_lambda x K_lambda, column-major): the rows of lambda of every ancestor basis U_tau,
//    then the dense blocks of lambda's rows.  With z_lambda = [u_t1; u_t2; ...; v|_s1; ...]
//    gathered into LDS, w|_lambda = B_lambda z_lambda: one lane per row (leaf size <= 64 =
//    wavefront size), each output element written exactly once, no atomics.  The user-order
//    permutation is folded into the gathers of v and the scatter of w.
//
// The H-matrix form uses the same forward / reduce / backward kernels with panels built
// from Y_b (forward, one segment per block) and X_b (backward).
//
// Every index the kernels use comes from arrays this file builds after validating the
// host image, so device accesses stay inside the allocations by construction.
#include "uhm_internal.h"

#include <mutex>

namespace uhm_detail {

thread_local std::string g_err;

const char* const kKernelNames[K_COUNT] = {
    "k_forward_tiles", "k_reduce_segments", "k_coupling", "k_reduce_coupling", "k_backward",
    "k_lp_gather", "k_lp_forward", "k_lp_reduce_segments", "k_lp_coupling", "k_lp_reduce_coupling",
    "k_lp_backward", "k_lp_scatter", "k_coupling_sym", "k_reduce_sym", "k_backward_sym", "k_finish_sym",
    "k_factor_in", "k_lp_factor_in"};

int check_tree(int64_t n, const int64_t* perm, int32_t nc, const int64_t* off, const int64_t* size,
               const int32_t* parent, TreeInfo& T) {
  if (n < 1 || n > INT32_MAX) return fail(UHM_EINVAL, "n must be in [1, 2^31)");
  if (!perm || !off || !size || !parent || nc < 1) return fail(UHM_EINVAL, "null cluster tree array");
  std::vector<char> seen(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (perm[i] < 0 || perm[i] >= n || seen[perm[i]]) return fail(UHM_EINVAL, "perm is not a permutation");
    seen[perm[i]] = 1;
  }
  int root = -1;
  std::vector<int32_t> nchild(nc, 0);
  for (int32_t c = 0; c < nc; ++c) {
    if (size[c] < 1 || off[c] < 0 || off[c] + size[c] > n) return fail(UHM_EINVAL, "cluster range out of [0, n)");
    if (parent[c] < 0) {
      if (root >= 0) return fail(UHM_EINVAL, "more than one root cluster");
      root = c;
      if (off[c] != 0 || size[c] != n) return fail(UHM_EINVAL, "root must cover [0, n)");
    } else {
      const int32_t p = parent[c];
      if (p >= nc || p == c) return fail(UHM_EINVAL, "bad parent index");
      if (off[c] < off[p] || off[c] + size[c] > off[p] + size[p]) return fail(UHM_EINVAL, "child outside parent");
      nchild[p]++;
    }
  }
  if (root < 0) return fail(UHM_EINVAL, "no root cluster");
  // children partition their parent
  std::vector<std::vector<int32_t>> kids(nc);
  for (int32_t c = 0; c < nc; ++c)
    if (parent[c] >= 0) kids[parent[c]].push_back(c);
  for (int32_t c = 0; c < nc; ++c) {
    if (kids[c].empty()) continue;
    std::sort(kids[c].begin(), kids[c].end(), [&](int32_t a, int32_t b) { return off[a] < off[b]; });
    int64_t pos = off[c];
    for (int32_t k : kids[c]) {
      if (off[k] != pos) return fail(UHM_EINVAL, "children do not partition their parent");
      pos += size[k];
    }
    if (pos != off[c] + size[c]) return fail(UHM_EINVAL, "children do not partition their parent");
  }
  T.n = n;
  T.nc = nc;
  for (int32_t c = 0; c < nc; ++c)
    if (nchild[c] == 0) T.leaves.push_back(c);
  std::sort(T.leaves.begin(), T.leaves.end(), [&](int32_t a, int32_t b) { return off[a] < off[b]; });
  int64_t pos = 0;
  for (int32_t l : T.leaves) {
    if (off[l] != pos) return fail(UHM_EINVAL, "leaves do not tile [0, n)");
    if (size[l] > kLeafMax) return fail(UHM_ENOTSUP, "leaf larger than 64 points");
    pos += size[l];
  }
  if (pos != n) return fail(UHM_EINVAL, "leaves do not tile [0, n)");
  const int32_t nl = (int32_t)T.leaves.size();
  std::vector<int64_t> loff(nl);
  for (int32_t i = 0; i < nl; ++i) loff[i] = off[T.leaves[i]];
  T.leaf_first.assign(nc, 0);
  T.leaf_cnt.assign(nc, 0);
  for (int32_t c = 0; c < nc; ++c) {
    const int32_t a = (int32_t)(std::lower_bound(loff.begin(), loff.end(), off[c]) - loff.begin());
    const int32_t b = (int32_t)(std::lower_bound(loff.begin(), loff.end(), off[c] + size[c]) - loff.begin());
    T.leaf_first[c] = a;
    T.leaf_cnt[c] = b - a;
  }
  T.anc.resize(nl);
  for (int32_t i = 0; i < nl; ++i) {
    std::vector<int32_t>& a = T.anc[i];
    int32_t c = T.leaves[i];
    int guard = 0;
    while (c >= 0) {
      a.push_back(c);
      c = parent[c];
      if (++guard > nc) return fail(UHM_EINVAL, "cycle in the parent array");
    }
    std::reverse(a.begin(), a.end());
  }
  return UHM_OK;
}

hipEvent_t get_event(uhm_op* op) {
  if (!op->free_events.empty()) {
    hipEvent_t e = op->free_events.back();
    op->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int common_tree_upload(uhm_op* op, const TreeInfo& T, const int64_t* perm, const int64_t* off, const int64_t* size,
                       hipStream_t s) {
  std::vector<int32_t> p32(T.n), ip32(T.n), lp(T.leaves.size()), ln(T.leaves.size());
  for (int64_t i = 0; i < T.n; ++i) {
    p32[i] = (int32_t)perm[i];
    ip32[perm[i]] = (int32_t)i;   // perm was checked to be a permutation
  }
  for (size_t i = 0; i < T.leaves.size(); ++i) {
    lp[i] = (int32_t)off[T.leaves[i]];
    ln[i] = (int32_t)size[T.leaves[i]];
  }
  int rc;
  if ((rc = op->perm.upload(p32, s)) || (rc = op->iperm.upload(ip32, s)) || (rc = op->leaf_pos.upload(lp, s)) ||
      (rc = op->leaf_n.upload(ln, s)))
    return rc;
  UHM_HIP(hipStreamSynchronize(s));
  op->n = T.n;
  op->nleaves = (int32_t)T.leaves.size();
  return UHM_OK;
}

}  // namespace uhm_detail

using namespace uhm_detail;

namespace {

// ------------------------------------------------------------------ device kernels

// Map workgroup ids so that each XCD (workgroups are dealt round-robin over 8 XCDs)
// receives a contiguous range of leaves: neighbouring leaves share ancestors, whose
// rank-space vectors then stay in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7, x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

// Streaming loads of operator data: each element is read once per product, so the loads
// carry the nontemporal hint and do not displace the reused vectors from the caches.
typedef double v2d_stream __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cd stream_load(const cd* p) {
  const v2d_stream v = __builtin_nontemporal_load(reinterpret_cast<const v2d_stream*>(p));
  return make_double2(v.x, v.y);
}

// Forward transform: one wave per 64-column tile of a leaf's panel (tiles listed leaf by
// leaf), lane c accumulating conj(F[i,c]) x_i over the leaf's rows i.  The leaf's x values
// are uniform over the wave and come through scalar loads.
template <int FORM>
__global__ __launch_bounds__(64 * kFwdWaves) void k_forward_tiles(
    const cd* __restrict__ F, const int2* __restrict__ ftiles, int32_t ntiles, const int64_t* __restrict__ fwd_off,
    const int32_t* __restrict__ fwd_cols, const int32_t* __restrict__ leaf_pos, const int32_t* __restrict__ leaf_n,
    const int32_t* __restrict__ perm, const cd* __restrict__ x, const int64_t* __restrict__ poff, cd* __restrict__ p) {
  const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * kFwdWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int2 lt = ftiles[tile];
  const int leaf = lt.x, j = lt.y;
  const int n = leaf_n[leaf];
  const int wj = min(kTile, fwd_cols[leaf] - kTile * j);
  if (lane >= wj) return;
  const cd* q = F + fwd_off[leaf] + (int64_t)kTile * j * n + lane;
  const int32_t* px = perm + leaf_pos[leaf];
  double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    cd v[8], xv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = stream_load(&q[(i + k) * wj]);
#pragma unroll
    for (int k = 0; k < 8; ++k) xv[k] = x[px[i + k]];
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      re0 = fma(v[k].x, xv[k].x, fma(v[k].y, xv[k].y, re0));
      im0 = fma(v[k].x, xv[k].y, fma(-v[k].y, xv[k].x, im0));
      re1 = fma(v[k + 1].x, xv[k + 1].x, fma(v[k + 1].y, xv[k + 1].y, re1));
      im1 = fma(v[k + 1].x, xv[k + 1].y, fma(-v[k + 1].y, xv[k + 1].x, im1));
    }
  }
  for (; i < n; ++i) {
    const cd v = stream_load(&q[i * wj]), xv = x[px[i]];
    re0 = fma(v.x, xv.x, fma(v.y, xv.y, re0));
    im0 = fma(v.x, xv.y, fma(-v.y, xv.x, im0));
  }
  p[poff[leaf] + kTile * j + lane] = make_double2(re0 + re1, im0 + im1);
}

// out[e] = sum over the leaves of segment seg(e) of p[leaf][col(seg) + e - start(seg)],
// leaves taken in cluster order.
template <int FORM>
__global__ __launch_bounds__(256) void k_reduce_segments(
    const cd* __restrict__ p, const int64_t* __restrict__ poff, const int32_t* __restrict__ out_seg,
    const int64_t* __restrict__ seg_start, const int32_t* __restrict__ seg_leaf0, const int32_t* __restrict__ seg_nleaf,
    const int32_t* __restrict__ seg_col, int64_t nout, cd* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  const int s = out_seg[e];
  const int col = seg_col[s] + (int)(e - seg_start[s]);
  const int l0 = seg_leaf0[s], nl = seg_nleaf[s];
  // fixed summation order (leaf order), eight independent loads in flight
  double re = 0.0, im = 0.0;
  int q = 0;
  for (; q + 8 <= nl; q += 8) {
    int64_t o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = poff[l0 + q + k];
    cd v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[o[k] + col];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      re += v[k].x;
      im += v[k].y;
    }
  }
  for (; q < nl; ++q) {
    const cd v = p[poff[l0 + q] + col];
    re += v.x;
    im += v.y;
  }
  out[e] = make_double2(re, im);
}



// part[tile][r] = sum_c S_chunk[r, c] * xh[src(c)] over the tile's columns.
__global__ __launch_bounds__(64 * kCoupWaves) void k_coupling(
    const cd* __restrict__ S, const CoupTile* __restrict__ tiles, int32_t ntiles, const int2* __restrict__ cblk,
    const cd* __restrict__ xh, cd* __restrict__ part) {
  // wave-uniform tile index: the descriptors and the rank-space values then come
  // through scalar loads
  const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * kCoupWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const CoupTile T = tiles[tile];
  double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
  const int h = T.h;
  const bool act = lane < h;
  const cd* col = S + T.s_base + (act ? lane : 0);
  int b = T.first_blk, j = T.first_col, rem = T.ncols;
  while (rem > 0) {
    const int2 bl = cblk[b];
    const int cnt = min(bl.x - j, rem);
    const cd* xv = xh + bl.y + j;
    int q = 0;
    for (; q + 8 <= cnt; q += 8) {
      cd sv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) sv[k] = stream_load(&col[(int64_t)(q + k) * h]);
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        const cd x0 = xv[q + k], x1 = xv[q + k + 1];
        re0 = fma(sv[k].x, x0.x, fma(-sv[k].y, x0.y, re0));
        im0 = fma(sv[k].x, x0.y, fma(sv[k].y, x0.x, im0));
        re1 = fma(sv[k + 1].x, x1.x, fma(-sv[k + 1].y, x1.y, re1));
        im1 = fma(sv[k + 1].x, x1.y, fma(sv[k + 1].y, x1.x, im1));
      }
    }
    for (; q < cnt; ++q) {
      const cd s0 = stream_load(&col[(int64_t)q * h]), x0 = xv[q];
      re0 = fma(s0.x, x0.x, fma(-s0.y, x0.y, re0));
      im0 = fma(s0.x, x0.y, fma(s0.y, x0.x, im0));
    }
    col += (int64_t)cnt * h;
    rem -= cnt;
    ++b;
    j = 0;
  }
  if (act) part[(int64_t)tile * kRowChunk + lane] = make_double2(re0 + re1, im0 + im1);
}

// First step of the factored couplings: out[t_out + c] = sum_r conj(FY[r, c]) u[x_row + r]
// over the l_sigma rows of one tile, one lane per column (t_b = S_{Y,b}^* u_sigma); u_sigma
// is uniform over the wave and comes through scalar loads.  u and out are the two disjoint
// parts of the coupling source vector ([0, nxh) and [nxh, nsrc)).
__global__ __launch_bounds__(64 * kCoupWaves) void k_factor_in(const cd* __restrict__ FY,
                                                               const FacTile* __restrict__ ftl, int32_t ntiles,
                                                               const cd* __restrict__ u_all,
                                                               cd* __restrict__ out) {
  const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * kCoupWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const FacTile T = ftl[tile];
  if (lane >= T.wj) return;
  const cd* q = FY + T.f_base + lane;
  const cd* u = u_all + T.x_row;
  const int wj = T.wj, n = T.rows;
  double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    cd v[8], uv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = stream_load(&q[(int64_t)(i + k) * wj]);
#pragma unroll
    for (int k = 0; k < 8; ++k) uv[k] = u[i + k];
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      re0 = fma(v[k].x, uv[k].x, fma(v[k].y, uv[k].y, re0));
      im0 = fma(v[k].x, uv[k].y, fma(-v[k].y, uv[k].x, im0));
      re1 = fma(v[k + 1].x, uv[k + 1].x, fma(v[k + 1].y, uv[k + 1].y, re1));
      im1 = fma(v[k + 1].x, uv[k + 1].y, fma(-v[k + 1].y, uv[k + 1].x, im1));
    }
  }
  for (; i < n; ++i) {
    const cd v = stream_load(&q[(int64_t)i * wj]), uv = u[i];
    re0 = fma(v.x, uv.x, fma(v.y, uv.y, re0));
    im0 = fma(v.x, uv.y, fma(-v.y, uv.x, im0));
  }
  out[T.t_out + lane] = make_double2(re0 + re1, im0 + im1);
}

// yh[e] = sum_{t in tiles of e's chunk} part[t][r(e)], tiles in column order.
__global__ __launch_bounds__(256) void k_reduce_coupling(
    const cd* __restrict__ part, const int32_t* __restrict__ yh_grp, const int64_t* __restrict__ grp_start,
    const int32_t* __restrict__ grp_t0, const int32_t* __restrict__ grp_nt, int64_t nout, cd* __restrict__ yh) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  const int g = yh_grp[e];
  const int r = (int)(e - grp_start[g]);
  const int t0 = grp_t0[g], nt = grp_nt[g];
  double re = 0.0, im = 0.0;
  for (int t = 0; t < nt; ++t) {
    const cd v = part[(int64_t)(t0 + t) * kRowChunk + r];
    re += v.x;
    im += v.y;
  }
  yh[e] = make_double2(re, im);
}

// w|_lambda = B_lambda z_lambda with z gathered from the rank-space vector (index >= 0)
// or from the user-order input (index = -1 - user index).
template <int FORM>
__global__ __launch_bounds__(64 * kBwdWaves) void k_backward(
    const cd* __restrict__ B, const int64_t* __restrict__ bwd_off, const int32_t* __restrict__ bwd_cols,
    const int64_t* __restrict__ zoff, const int32_t* __restrict__ zmap, const int32_t* __restrict__ leaf_pos,
    const int32_t* __restrict__ leaf_n, const int32_t* __restrict__ perm, const cd* __restrict__ yh,
    const cd* __restrict__ x, cd* __restrict__ y, int nleaves) {
  const int leaf = xcd_remap(blockIdx.x, nleaves);
  const int K = bwd_cols[leaf], n = leaf_n[leaf];
  __shared__ cd zs[kBwdChunk];
  __shared__ cd red[kBwdWaves][kLeafMax];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const cd* Bl = B + bwd_off[leaf];
  const int32_t* zm = zmap + zoff[leaf];
  double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
  const bool act = lane < n;
  for (int c0 = 0; c0 < K; c0 += kBwdChunk) {
    const int cn = min(kBwdChunk, K - c0);
    __syncthreads();
    for (int c = t; c < cn; c += 64 * kBwdWaves) {
      const int m = zm[c0 + c];
      zs[c] = m >= 0 ? yh[m] : x[-1 - m];
    }
    __syncthreads();
    const int per = (cn + kBwdWaves - 1) / kBwdWaves;
    const int a = w * per, e = min(cn, a + per);
    if (act) {
      const cd* col = Bl + (int64_t)(c0 + a) * n + lane;
      int c = a;
      for (; c + 8 <= e; c += 8, col += 8 * n) {
        cd bv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) bv[k] = stream_load(&col[k * n]);
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
          const cd z0 = zs[c + k], z1 = zs[c + k + 1];
          re0 = fma(bv[k].x, z0.x, fma(-bv[k].y, z0.y, re0));
          im0 = fma(bv[k].x, z0.y, fma(bv[k].y, z0.x, im0));
          re1 = fma(bv[k + 1].x, z1.x, fma(-bv[k + 1].y, z1.y, re1));
          im1 = fma(bv[k + 1].x, z1.y, fma(bv[k + 1].y, z1.x, im1));
        }
      }
      for (; c < e; ++c, col += n) {
        const cd b0 = stream_load(col), z0 = zs[c];
        re0 = fma(b0.x, z0.x, fma(-b0.y, z0.y, re0));
        im0 = fma(b0.x, z0.y, fma(b0.y, z0.x, im0));
      }
    }
  }
  red[w][lane] = make_double2(re0 + re1, im0 + im1);
  __syncthreads();
  if (w == 0 && act) {
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < kBwdWaves; ++q) {
      sr += red[q][lane].x;
      si += red[q][lane].y;
    }
    y[perm[leaf_pos[leaf] + lane]] = make_double2(sr, si);
  }
}

// ------------------------------------------------------------------ symmetric storage
//
// Remark 4.4: rows and columns share one cluster set, V_sigma = conj(U_sigma), and only one
// block b = tau x sigma of each mirrored pair is stored; its mirror is applied as
// U_sigma S_b^T U_tau^T (admissible) or A|_b^T (dense).  Each stored element is read once
// and used twice: for the direct product (one lane per row, as above) and for the
// transposed one, whose column sums run across the 64 lanes of the wave.

constexpr int kSymBwdWaves = 8;
constexpr int kSymBwdChunk = 1024;  // z entries staged in LDS per round

__device__ __forceinline__ cd cmul(cd a, cd b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// x + y after swapping lanes 32-63 of x with lanes 0-31 of y (v_permlane32_swap): lanes
// 0-31 get x_L + x_{L+32}, lanes 32-63 get y_{L-32} + y_L.
__device__ __forceinline__ double swap32_add(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// The same with the odd 16-lane rows of x and the even rows of y (v_permlane16_swap):
// rows 0 and 2 get x_L + x_{L+16}, rows 1 and 3 get y_{L-16} + y_L.
__device__ __forceinline__ double swap16_add(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}

// A DPP lane move within 16-lane rows (CTRL: 0x11n = from lane L - n, 0x12n = from lane
// (L + n) mod 16 of the row); lanes whose source lies outside the row get 0.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Column sums of eight columns at once, all 64 lanes taking part.  p[k] is this lane's
// term of column k.  Three exchange steps halve the number of values per lane (lanes
// 0-31 keep columns 0-3 and 32-63 columns 4-7, then the 16-lane rows, then the 8-lane
// halves of a row), each adding the partner lane's terms of the kept columns; three
// shifted adds then sum the eight lanes that hold one column.  On return, lane L with
// (L & 7) == 7 holds the sum of column L >> 3.  Lane moves only (no LDS); the order of the
// additions is fixed, so the sums do not change from run to run.
__device__ __forceinline__ cd wave_colsum8(const cd (&p)[8], int lane) {
  cd q[4], r[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = make_double2(swap32_add(p[i].x, p[i + 4].x), swap32_add(p[i].y, p[i + 4].y));
#pragma unroll
  for (int i = 0; i < 2; ++i) r[i] = make_double2(swap16_add(q[i].x, q[i + 2].x), swap16_add(q[i].y, q[i + 2].y));
  const bool b3 = lane & 8;
  const cd keep = b3 ? r[1] : r[0], send = b3 ? r[0] : r[1];
  cd v = make_double2(keep.x + dpp_move<0x128>(send.x), keep.y + dpp_move<0x128>(send.y));  // row_ror:8 = lane ^ 8
  v = make_double2(v.x + dpp_move<0x111>(v.x), v.y + dpp_move<0x111>(v.y));                // row_shr:1
  v = make_double2(v.x + dpp_move<0x112>(v.x), v.y + dpp_move<0x112>(v.y));                // row_shr:2
  return make_double2(v.x + dpp_move<0x114>(v.x), v.y + dpp_move<0x114>(v.y));             // row_shr:4
}

// Direct:     part[tile][r]     = sum_c S_chunk[r, c] xh[csrc[c]]   (S_b u_sigma)
// Transposed: tpart[t_base + c] = sum_r S_chunk[r, c] xh[x_row + r] (S_b^T u_tau, this chunk's rows)
__global__ __launch_bounds__(64 * kCoupWaves) void k_coupling_sym(
    const cd* __restrict__ S, const SymTile* __restrict__ tiles, int32_t ntiles, const int32_t* __restrict__ csrc,
    const cd* __restrict__ xh, cd* __restrict__ part, cd* __restrict__ tpart) {
  const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * kCoupWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const SymTile T = tiles[tile];
  const int h = T.h;
  const bool act = lane < h;
  // lanes past the chunk read row 0 and weigh it by zero
  const cd xt = act ? xh[T.x_row + lane] : make_double2(0.0, 0.0);
  const cd* col = S + T.s_base + (act ? lane : 0);
  const int32_t* cs = csrc + T.c_base;
  // the column sums are collected in LDS and written out once per tile, in full lines:
  // small scattered writes in the middle of the operator stream cost far more than
  // their bytes
  __shared__ cd tbuf[kCoupWaves][kCoupCols];
  cd* tb = tbuf[threadIdx.x >> 6];
  double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
  const int nc = T.ncols;
  // groups of 8 columns, the next group's loads issued before this group's arithmetic;
  // the last group may run past the tile: the S array and the column-source table carry
  // slack for it, and the extra columns get a zero weight
  cd sv[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) sv[k] = stream_load(&col[(int64_t)k * h]);
  for (int q = 0; q < nc; q += 8) {
    const int rem = nc - q;
    cd xv[8], nx[8];
    if (q + 8 < nc) {
#pragma unroll
      for (int k = 0; k < 8; ++k) nx[k] = stream_load(&col[(int64_t)(q + 8 + k) * h]);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const cd v = xh[cs[q + k]];
      xv[k] = k < rem ? v : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      re0 = fma(sv[k].x, xv[k].x, fma(-sv[k].y, xv[k].y, re0));
      im0 = fma(sv[k].x, xv[k].y, fma(sv[k].y, xv[k].x, im0));
      re1 = fma(sv[k + 1].x, xv[k + 1].x, fma(-sv[k + 1].y, xv[k + 1].y, re1));
      im1 = fma(sv[k + 1].x, xv[k + 1].y, fma(sv[k + 1].y, xv[k + 1].x, im1));
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) sv[k] = cmul(sv[k], xt);
    const cd t = wave_colsum8(sv, lane);
    if ((lane & 7) == 7 && (lane >> 3) < rem) tb[q + (lane >> 3)] = t;
#pragma unroll
    for (int k = 0; k < 8; ++k) sv[k] = nx[k];
  }
  if (act) part[(int64_t)tile * kRowChunk + lane] = make_double2(re0 + re1, im0 + im1);
  // LDS operations of one wave complete in order; the barrier keeps the compiler from
  // moving the reads above the writes of other lanes
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  cd* tp = tpart + T.t_base;
  for (int c = lane; c < nc; c += 64) tp[c] = tb[c];
}

// yh[e] = (direct tiles of e's row chunk, in column order) + (transposed partials of the
// mirrored blocks, in table order).
__global__ __launch_bounds__(256) void k_reduce_sym(
    const cd* __restrict__ part, const cd* __restrict__ tpart, const int32_t* __restrict__ yh_grp,
    const int64_t* __restrict__ grp_start, const int32_t* __restrict__ grp_t0, const int32_t* __restrict__ grp_nt,
    const int32_t* __restrict__ grp_s0, const int32_t* __restrict__ grp_ns, const int64_t* __restrict__ tsrc,
    int64_t nout, cd* __restrict__ yh) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  const int g = yh_grp[e];
  const int r = (int)(e - grp_start[g]);
  const int t0 = grp_t0[g], nt = grp_nt[g], s0 = grp_s0[g], ns = grp_ns[g];
  double re = 0.0, im = 0.0;
  for (int t = 0; t < nt; ++t) {
    const cd v = part[(int64_t)(t0 + t) * kRowChunk + r];
    re += v.x;
    im += v.y;
  }
  int k = 0;
  for (; k + 4 <= ns; k += 4) {
    cd v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = tpart[tsrc[s0 + k + j] + r];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      re += v[j].x;
      im += v[j].y;
    }
  }
  for (; k < ns; ++k) {
    const cd v = tpart[tsrc[s0 + k] + r];
    re += v.x;
    im += v.y;
  }
  yh[e] = make_double2(re, im);
}

// As k_backward, and for the panel columns c >= tcol (stored off-diagonal dense blocks
// A|_b, b = lambda' x sigma with lambda inside lambda') also the column sums
// td[td_off + c - tcol] = sum_i B[i, c] v_i over the leaf's rows i: lambda's share of
// (A|_b^T v|_lambda').
__global__ __launch_bounds__(64 * kSymBwdWaves) void k_backward_sym(
    const cd* __restrict__ B, const int64_t* __restrict__ bwd_off, const int32_t* __restrict__ bwd_cols,
    const int32_t* __restrict__ bwd_tcol, const int64_t* __restrict__ td_off, const int64_t* __restrict__ zoff,
    const int32_t* __restrict__ zmap, const int32_t* __restrict__ leaf_pos, const int32_t* __restrict__ leaf_n,
    const int32_t* __restrict__ perm, const cd* __restrict__ yh, const cd* __restrict__ x, cd* __restrict__ y,
    cd* __restrict__ td, int nleaves) {
  const int leaf = xcd_remap(blockIdx.x, nleaves);
  const int K = bwd_cols[leaf], n = leaf_n[leaf], tc = bwd_tcol[leaf];
  __shared__ cd zs[kSymBwdChunk];
  __shared__ cd tdb[kSymBwdChunk];  // column sums of the chunk, written out in full lines
  __shared__ cd red[kSymBwdWaves][kLeafMax];
  // the wave index is uniform over the wave: the column loop then branches on scalars
  const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
  const cd* Bl = B + bwd_off[leaf];
  const int32_t* zm = zmap + zoff[leaf];
  cd* tdl = td + td_off[leaf];
  const bool act = lane < n;
  const cd xr = act ? x[perm[leaf_pos[leaf] + lane]] : make_double2(0.0, 0.0);
  double re0 = 0.0, im0 = 0.0, re1 = 0.0, im1 = 0.0;
  for (int c0 = 0; c0 < K; c0 += kSymBwdChunk) {
    const int cn = min(kSymBwdChunk, K - c0);
    __syncthreads();
    // z of this chunk, then zeros up to the next multiple of 8 columns
    for (int c = t; c < ((cn + 7) & ~7); c += 64 * kSymBwdWaves) {
      if (c < cn) {
        const int m = zm[c0 + c];
        zs[c] = m >= 0 ? yh[m] : x[-1 - m];
      } else {
        zs[c] = make_double2(0.0, 0.0);
      }
    }
    __syncthreads();
    // groups of 8 columns dealt round-robin to the waves; the last group of the chunk
    // may run past it (into the next chunk, or the slack after the last panel), where
    // the zero z entries take the extra columns out of the direct product
    for (int c = 8 * w; c < cn; c += 8 * kSymBwdWaves) {
      const cd* col = Bl + (int64_t)(c0 + c) * n + (act ? lane : 0);
      cd bv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) bv[k] = stream_load(&col[k * n]);
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        const cd z0 = zs[c + k], z1 = zs[c + k + 1];
        re0 = fma(bv[k].x, z0.x, fma(-bv[k].y, z0.y, re0));
        im0 = fma(bv[k].x, z0.y, fma(bv[k].y, z0.x, im0));
        re1 = fma(bv[k + 1].x, z1.x, fma(-bv[k + 1].y, z1.y, re1));
        im1 = fma(bv[k + 1].x, z1.y, fma(bv[k + 1].y, z1.x, im1));
      }
      const int g = c0 + c;  // panel column of bv[0]
      if (g + 8 > tc) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const cd xk = g + k >= tc ? xr : make_double2(0.0, 0.0);
          bv[k] = cmul(bv[k], xk);
        }
        const cd s = wave_colsum8(bv, lane);
        const int kk = lane >> 3;
        if ((lane & 7) == 7 && c + kk < cn && g + kk >= tc) tdb[c + kk] = s;
      }
    }
    if (c0 + cn > tc) {  // uniform over the workgroup
      __syncthreads();
      for (int c = max(c0, tc) - c0 + t; c < cn; c += 64 * kSymBwdWaves) tdl[c0 + c - tc] = tdb[c];
    }
  }
  red[w][lane] = make_double2(re0 + re1, im0 + im1);
  __syncthreads();
  if (w == 0 && act) {
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < kSymBwdWaves; ++q) {
      sr += red[q][lane].x;
      si += red[q][lane].y;
    }
    y[perm[leaf_pos[leaf] + lane]] = make_double2(sr, si);
  }
}

// w|_mu += sum of the transposed dense partials addressed to leaf mu, in table order.
__global__ __launch_bounds__(64) void k_finish_sym(
    const int32_t* __restrict__ fin_off, const int32_t* __restrict__ fin_cnt, const int64_t* __restrict__ fsrc,
    const int32_t* __restrict__ leaf_pos, const int32_t* __restrict__ leaf_n, const int32_t* __restrict__ perm,
    const cd* __restrict__ td, cd* __restrict__ y) {
  const int leaf = blockIdx.x, lane = threadIdx.x;
  const int cnt = fin_cnt[leaf];
  if (cnt == 0 || lane >= leaf_n[leaf]) return;
  const int64_t* src = fsrc + fin_off[leaf];
  const int idx = perm[leaf_pos[leaf] + lane];
  cd acc = y[idx];
  for (int k = 0; k < cnt; ++k) {
    const cd v = td[src[k] + lane];
    acc.x += v.x;
    acc.y += v.y;
  }
  y[idx] = acc;
}

// ------------------------------------------------------------------ host structures

// A column source of a forward or backward panel: `len` columns of a column-major
// matrix `src` (rows `nrows`), starting at row `row0` for this leaf.
struct PanelSeg {
  const cd* src;
  int64_t nrows;
  int64_t row0;
  int32_t len;
  int32_t zbase;  // backward: rank-space index of the first column, or -1 for dense
  const int64_t* dense_cols;  // backward dense: perm + off[sigma]
  bool conj = false;          // forward: store the complex conjugate
};

// Forward panel of one leaf: tile-major, tiles of 64 columns, each row-major.
int stage_forward_leaf(Stager& st, const std::vector<PanelSeg>& segs, int32_t C, int32_t n) {
  // column c -> (segment, column within segment)
  std::vector<std::pair<int32_t, int32_t>> cmap;
  cmap.reserve(C);
  for (int32_t si = 0; si < (int32_t)segs.size(); ++si)
    for (int32_t j = 0; j < segs[si].len; ++j) cmap.push_back({si, j});
  for (int32_t j0 = 0; j0 < C; j0 += kTile) {
    const int32_t wj = std::min(kTile, C - j0);
    cd* tile = st.span((int64_t)wj * n);
    for (int32_t c = 0; c < wj; ++c) {
      const PanelSeg& sg = segs[cmap[j0 + c].first];
      const cd* colp = sg.src + (int64_t)cmap[j0 + c].second * sg.nrows + sg.row0;
      if (sg.conj)
        for (int32_t i = 0; i < n; ++i) tile[(int64_t)i * wj + c] = make_double2(colp[i].x, -colp[i].y);
      else
        for (int32_t i = 0; i < n; ++i) tile[(int64_t)i * wj + c] = colp[i];
    }
  }
  return st.err;
}

// Backward panel of one leaf: column-major n x K.
int stage_backward_leaf(Stager& st, const std::vector<PanelSeg>& segs, int32_t n) {
  for (const PanelSeg& sg : segs)
    for (int32_t j = 0; j < sg.len; ++j) {
      cd* dst = st.span(n);
      std::memcpy(static_cast<void*>(dst), sg.src + (int64_t)j * sg.nrows + sg.row0, sizeof(cd) * (size_t)n);
    }
  return st.err;
}

struct SegDesc {
  int64_t start;
  int32_t len;
  int32_t leaf0, nleaf, col;
};

int upload_segments(uhm_op* op, const std::vector<SegDesc>& segs, int64_t nout, hipStream_t s) {
  std::vector<int32_t> out_seg(nout), leaf0(segs.size()), nleaf(segs.size()), col(segs.size());
  std::vector<int64_t> start(segs.size());
  for (size_t k = 0; k < segs.size(); ++k) {
    for (int32_t j = 0; j < segs[k].len; ++j) out_seg[segs[k].start + j] = (int32_t)k;
    start[k] = segs[k].start;
    leaf0[k] = segs[k].leaf0;
    nleaf[k] = segs[k].nleaf;
    col[k] = segs[k].col;
  }
  int rc;
  if ((rc = op->out_seg.upload(out_seg, s)) || (rc = op->seg_start.upload(start, s)) ||
      (rc = op->seg_leaf0.upload(leaf0, s)) || (rc = op->seg_nleaf.upload(nleaf, s)) ||
      (rc = op->seg_col.upload(col, s)))
    return rc;
  UHM_HIP(hipStreamSynchronize(s));
  op->nxh = nout;
  return UHM_OK;
}

// (leaf, tile) list of the 64-column tiles of the forward panels, leaf by leaf.
int upload_fwd_tiles(uhm_op* op, const std::vector<int32_t>& fwd_cols, hipStream_t s) {
  std::vector<int2> t;
  for (size_t i = 0; i < fwd_cols.size(); ++i)
    for (int32_t j = 0; j * kTile < fwd_cols[i]; ++j) t.push_back(make_int2((int)i, j));
  if (t.size() > (size_t)INT32_MAX) return fail(UHM_ENOTSUP, "too many forward tiles");
  op->nftiles = (int32_t)t.size();
  return op->ftiles.upload(t, s);
}

struct FwdLayout {
  int64_t ftot = 0, ptot = 0;
  std::vector<int64_t> fwd_off, poff;
  std::vector<int32_t> fwd_cols;
  std::vector<SegDesc> segs;
};

// Forward panels of the bases W_c (size[c] x rank[c] at W + W_off[c], conjugated on the
// way if `conj`) of every cluster with rank[c] > 0, and the segment tables that add the
// per-leaf partial sums into u_c = W_c^* v|_c at xh_off[c].
int build_forward(uhm_op* op, const TreeInfo& T, const int64_t* off, const int64_t* size, const int32_t* rank,
                  const cd* W, const int64_t* W_off, bool conj, const std::vector<int64_t>& xh_off, int64_t nxh,
                  hipStream_t s, FwdLayout& L) {
  const int32_t nl = (int32_t)T.leaves.size(), nc = T.nc;
  L.fwd_off.assign(nl, 0);
  L.poff.assign(nl, 0);
  L.fwd_cols.assign(nl, 0);
  std::vector<int32_t> seg_col_of(nc, -1);  // column of cluster c's segment in its leaves' panels
  int64_t ftot = 0, ptot = 0;
  for (int32_t i = 0; i < nl; ++i) {
    int32_t C = 0;
    for (int32_t a : T.anc[i])
      if (rank[a] > 0) {
        if (seg_col_of[a] < 0) seg_col_of[a] = C;
        C += rank[a];
      }
    L.fwd_cols[i] = C;
    L.fwd_off[i] = ftot;
    L.poff[i] = ptot;
    ftot += (int64_t)C * size[T.leaves[i]];
    ptot += C;
  }
  int rc;
  if ((rc = op->F.alloc(ftot))) return rc;
  {
    Stager st;
    if ((rc = st.init(op->F.p, ftot, s))) return rc;
    std::vector<PanelSeg> segs;
    for (int32_t i = 0; i < nl && !st.err; ++i) {
      const int32_t lf = T.leaves[i];
      segs.clear();
      for (int32_t a : T.anc[i])
        if (rank[a] > 0) segs.push_back({W + W_off[a], size[a], off[lf] - off[a], rank[a], -1, nullptr, conj});
      if ((rc = stage_forward_leaf(st, segs, L.fwd_cols[i], (int32_t)size[lf]))) return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = op->fwd_off.upload(L.fwd_off, s)) || (rc = op->fwd_cols.upload(L.fwd_cols, s)) ||
      (rc = op->poff.upload(L.poff, s)) || (rc = upload_fwd_tiles(op, L.fwd_cols, s)))
    return rc;
  op->p_len = ptot;
  L.ftot = ftot;
  L.ptot = ptot;
  L.segs.clear();
  for (int32_t c = 0; c < nc; ++c)
    if (rank[c] > 0) L.segs.push_back({xh_off[c], rank[c], T.leaf_first[c], T.leaf_cnt[c], seg_col_of[c]});
  return upload_segments(op, L.segs, nxh, s);
}


int grow_workspace(uhm_op* op) {
  // single-RHS workspace; columns are processed one at a time
  int rc;
  if (op->ws_p.n < op->p_len && (rc = op->ws_p.alloc(op->p_len))) return rc;
  const int64_t nsrc = std::max(op->nxh, op->nsrc);
  if (op->ws_xh.n < nsrc && (rc = op->ws_xh.alloc(nsrc))) return rc;
  if (op->kind == 0) {
    if (op->ws_part.n < (int64_t)op->nctiles * kRowChunk && (rc = op->ws_part.alloc((int64_t)op->nctiles * kRowChunk)))
      return rc;
    if (op->ws_yh.n < op->nyh && (rc = op->ws_yh.alloc(op->nyh))) return rc;
  }
  if (op->sym) {
    if (op->ws_tpart.n < op->ttot && (rc = op->ws_tpart.alloc(op->ttot))) return rc;
    if (op->ws_td.n < op->tdtot && (rc = op->ws_td.alloc(op->tdtot))) return rc;
  }
  return UHM_OK;
}

// Host check of every index the kernels form, against the sizes of the arrays they
// touch.  Runs at the end of each upload, before the operator can be launched.
struct LayoutView {
  int64_t n, nleaves, ftot, ptot, btot, ztot, nz, nxh;
  const std::vector<int32_t>* leaf_n;
  const std::vector<int64_t>* fwd_off;
  const std::vector<int32_t>* fwd_cols;
  const std::vector<int64_t>* poff;
  const std::vector<SegDesc>* segs;
  const std::vector<int64_t>* bwd_off;
  const std::vector<int32_t>* bwd_cols;
  const std::vector<int64_t>* zoff;
  const std::vector<int32_t>* zmap;
};

int check_layout(const LayoutView& L) {
  for (int64_t i = 0; i < L.nleaves; ++i) {
    const int64_t n = (*L.leaf_n)[i], C = (*L.fwd_cols)[i], K = (*L.bwd_cols)[i];
    if (n < 1 || n > kLeafMax) return fail(UHM_EINVAL, "layout: leaf size");
    if ((*L.fwd_off)[i] < 0 || (*L.fwd_off)[i] + C * n > L.ftot) return fail(UHM_EINVAL, "layout: forward panel");
    if ((*L.poff)[i] < 0 || (*L.poff)[i] + C > L.ptot) return fail(UHM_EINVAL, "layout: partial sums");
    if ((*L.bwd_off)[i] < 0 || (*L.bwd_off)[i] + K * n > L.btot) return fail(UHM_EINVAL, "layout: backward panel");
    if ((*L.zoff)[i] < 0 || (*L.zoff)[i] + K > L.ztot) return fail(UHM_EINVAL, "layout: gather map");
  }
  for (const SegDesc& sg : *L.segs) {
    if (sg.start < 0 || sg.start + sg.len > L.nxh || sg.leaf0 < 0 || sg.nleaf < 1 || sg.leaf0 + sg.nleaf > L.nleaves)
      return fail(UHM_EINVAL, "layout: segment");
    for (int32_t q = 0; q < sg.nleaf; ++q)
      if (sg.col < 0 || sg.col + sg.len > (*L.fwd_cols)[sg.leaf0 + q]) return fail(UHM_EINVAL, "layout: segment column");
  }
  for (int32_t m : *L.zmap)
    if (m >= L.nz || (m < 0 && -1 - (int64_t)m >= L.n)) return fail(UHM_EINVAL, "layout: gather index");
  return UHM_OK;
}

int check_coupling(const std::vector<CoupTile>& tiles, const std::vector<int2>& cblk, int64_t stot, int64_t nxh,
                   const std::vector<int32_t>& grp_t0, const std::vector<int32_t>& grp_nt,
                   const std::vector<int64_t>& grp_start, int64_t nyh) {
  for (const int2& b : cblk)
    if (b.x < 1 || b.y < 0 || (int64_t)b.y + b.x > nxh) return fail(UHM_EINVAL, "layout: coupling block");
  for (const CoupTile& T : tiles) {
    if (T.h < 1 || T.h > kRowChunk || T.ncols < 1 || T.s_base < 0 || T.s_base + (int64_t)T.ncols * T.h > stot)
      return fail(UHM_EINVAL, "layout: coupling tile");
    int64_t b = T.first_blk, j = T.first_col, rem = T.ncols;
    while (rem > 0) {
      if (b < 0 || b >= (int64_t)cblk.size() || j < 0 || j >= cblk[b].x) return fail(UHM_EINVAL, "layout: coupling walk");
      rem -= std::min<int64_t>(cblk[b].x - j, rem);
      ++b;
      j = 0;
    }
  }
  for (size_t g = 0; g < grp_t0.size(); ++g) {
    if (grp_t0[g] < 0 || grp_nt[g] < 1 || (size_t)grp_t0[g] + grp_nt[g] > tiles.size())
      return fail(UHM_EINVAL, "layout: coupling group");
    const int32_t h = tiles[grp_t0[g]].h;
    if (grp_start[g] < 0 || grp_start[g] + h > nyh) return fail(UHM_EINVAL, "layout: coupling group rows");
  }
  return UHM_OK;
}


// Elements of zeros after the symmetric form's couplings and backward panels: a group of
// 8 columns that starts inside a tile (or panel range) may read 7 columns past its end.
constexpr int64_t kSymSlack = 8 * kLeafMax;
static_assert(kRowChunk <= kLeafMax, "slack covers 8 coupling columns too");

// Index checks of the symmetric-storage tables, against the sizes of the arrays the
// kernels touch (the couplings and panels have kSymSlack elements after stot and btot).
int check_sym(const std::vector<SymTile>& tiles, int64_t stot, int64_t ttot, const std::vector<int32_t>& csrc,
              int64_t nrs, const std::vector<int64_t>& grp_start, const std::vector<int32_t>& grp_t0,
              const std::vector<int32_t>& grp_nt, const std::vector<int32_t>& grp_s0,
              const std::vector<int32_t>& grp_ns, const std::vector<int64_t>& tsrc, const std::vector<int32_t>& leaf_n,
              const std::vector<int32_t>& bwd_cols, const std::vector<int32_t>& bwd_tcol,
              const std::vector<int64_t>& td_off, int64_t tdtot, const std::vector<int32_t>& fin_off,
              const std::vector<int32_t>& fin_cnt, const std::vector<int64_t>& fsrc) {
  for (const SymTile& T : tiles) {
    if (T.h < 1 || T.h > kRowChunk || T.ncols < 1 || T.s_base < 0 || T.s_base + (int64_t)T.ncols * T.h > stot ||
        T.t_base < 0 || T.t_base + T.ncols > ttot || T.c_base < 0 ||
        (int64_t)T.c_base + T.ncols + 7 > (int64_t)csrc.size() ||
        T.x_row < 0 || (int64_t)T.x_row + T.h > nrs)
      return fail(UHM_EINVAL, "layout: symmetric coupling tile");
  }
  for (int32_t c : csrc)
    if (c < 0 || c >= nrs) return fail(UHM_EINVAL, "layout: symmetric column source");
  const size_t ng = grp_start.size();
  std::vector<int32_t> gh(ng, 0);
  for (size_t g = 0; g < ng; ++g) {
    const int64_t end = g + 1 < ng ? grp_start[g + 1] : nrs;
    gh[g] = (int32_t)(end - grp_start[g]);
    if (grp_start[g] < 0 || gh[g] < 1 || gh[g] > kRowChunk || grp_nt[g] < 0 || grp_t0[g] < 0 ||
        (size_t)grp_t0[g] + grp_nt[g] > tiles.size() || grp_ns[g] < 0 || grp_s0[g] < 0 ||
        (size_t)grp_s0[g] + grp_ns[g] > tsrc.size())
      return fail(UHM_EINVAL, "layout: symmetric group");
    for (int32_t t = 0; t < grp_nt[g]; ++t)
      if (tiles[grp_t0[g] + t].h < gh[g]) return fail(UHM_EINVAL, "layout: symmetric group rows");
    for (int32_t k = 0; k < grp_ns[g]; ++k)
      if (tsrc[grp_s0[g] + k] < 0 || tsrc[grp_s0[g] + k] + gh[g] > ttot)
        return fail(UHM_EINVAL, "layout: symmetric transposed source");
  }
  const size_t nl = leaf_n.size();
  for (size_t i = 0; i < nl; ++i) {
    if (bwd_tcol[i] < 0 || bwd_tcol[i] > bwd_cols[i] || td_off[i] < 0 ||
        td_off[i] + (bwd_cols[i] - bwd_tcol[i]) > tdtot)
      return fail(UHM_EINVAL, "layout: symmetric near field");
    if (fin_cnt[i] < 0 || fin_off[i] < 0 || (size_t)fin_off[i] + fin_cnt[i] > fsrc.size())
      return fail(UHM_EINVAL, "layout: symmetric finish table");
    for (int32_t k = 0; k < fin_cnt[i]; ++k)
      if (fsrc[fin_off[i] + k] < 0 || fsrc[fin_off[i] + k] + leaf_n[i] > tdtot)
        return fail(UHM_EINVAL, "layout: symmetric finish source");
  }
  return UHM_OK;
}

// Upload of the symmetric storage form (Remark 4.4).  The image lists one block of each
// mirrored pair; U is the one cluster basis (V_c = conj(U_c) is implied and V, V_off and
// rank_col are not read).
int upload_sym(const uhm_host_operator* h, hipStream_t s, const TreeInfo& T, uhm_op* op) {
  const int32_t nc = h->nclusters;
  if (!h->rank_row || !h->U_off) return fail(UHM_EINVAL, "null basis arrays");
  if ((h->nadm > 0 && (!h->adm_row || !h->adm_col || !h->S_off || !h->S)) ||
      (h->nden > 0 && (!h->den_row || !h->den_col || !h->D_off || !h->D)) || h->nadm < 0 || h->nden < 0)
    return fail(UHM_EINVAL, "null block arrays");
  const int32_t* rank = h->rank_row;
  for (int32_t c = 0; c < nc; ++c) {
    if (rank[c] < 0 || rank[c] > h->size[c]) return fail(UHM_EINVAL, "cluster rank out of range");
    if (rank[c] > 0 && (!h->U || !in_bounds(h->U_off[c], h->size[c] * rank[c], h->U_len)))
      return fail(UHM_EINVAL, "U_off out of bounds");
  }
  std::vector<std::pair<int32_t, int32_t>> pairs;
  for (int64_t b = 0; b < h->nadm; ++b) {
    const int32_t t = h->adm_row[b], sg = h->adm_col[b];
    if (t < 0 || t >= nc || sg < 0 || sg >= nc) return fail(UHM_EINVAL, "admissible block cluster out of range");
    if (t == sg) return fail(UHM_EINVAL, "symmetric storage: a diagonal admissible block");
    if (rank[t] < 1 || rank[sg] < 1) return fail(UHM_EINVAL, "admissible block without bases");
    if (!in_bounds(h->S_off[b], (int64_t)rank[t] * rank[sg], h->S_len)) return fail(UHM_EINVAL, "S_off out of bounds");
    pairs.push_back({std::min(t, sg), std::max(t, sg)});
  }
  std::sort(pairs.begin(), pairs.end());
  if (std::adjacent_find(pairs.begin(), pairs.end()) != pairs.end())
    return fail(UHM_EINVAL, "symmetric storage: a block and its mirror (or a block twice) are both listed");
  pairs.clear();
  for (int64_t b = 0; b < h->nden; ++b) {
    const int32_t t = h->den_row[b], sg = h->den_col[b];
    if (t < 0 || t >= nc || sg < 0 || sg >= nc) return fail(UHM_EINVAL, "dense block cluster out of range");
    if (!in_bounds(h->D_off[b], h->size[t] * h->size[sg], h->D_len)) return fail(UHM_EINVAL, "D_off out of bounds");
    pairs.push_back({std::min(t, sg), std::max(t, sg)});
  }
  std::sort(pairs.begin(), pairs.end());
  if (std::adjacent_find(pairs.begin(), pairs.end()) != pairs.end())
    return fail(UHM_EINVAL, "symmetric storage: a dense block and its mirror (or a block twice) are both listed");

  const int32_t nl = op->nleaves;
  const cd* U = reinterpret_cast<const cd*>(h->U);
  const cd* Sh = reinterpret_cast<const cd*>(h->S);
  const cd* D = reinterpret_cast<const cd*>(h->D);
  int rc;

  // ---- one rank-space vector: u_c (forward) and its coupling result share offsets
  std::vector<int64_t> rs_off(nc, -1);
  int64_t nrs = 0;
  for (int32_t c = 0; c < nc; ++c)
    if (rank[c] > 0) { rs_off[c] = nrs; nrs += rank[c]; }
  if (nrs > INT32_MAX) return fail(UHM_ENOTSUP, "rank space too large");

  // ---- forward: u_c = conj(U_c)^* v|_c = U_c^T v|_c
  FwdLayout FL;
  if ((rc = build_forward(op, T, h->off, h->size, rank, U, h->U_off, true, rs_off, nrs, s, FL))) return rc;

  // ---- couplings of the stored blocks, by row cluster, in row chunks
  std::vector<std::vector<int64_t>> rowblk(nc), colblk(nc);
  for (int64_t b = 0; b < h->nadm; ++b) {
    rowblk[h->adm_row[b]].push_back(b);
    colblk[h->adm_col[b]].push_back(b);
  }
  std::vector<int32_t> colstart(h->nadm, 0);                    // first column of b in [S_b1 S_b2 ...]
  std::vector<std::vector<int64_t>> chunk_tp(nc);               // transposed-partial base per row chunk
  std::vector<std::vector<std::pair<int32_t, int32_t>>> chunk_tiles(nc);  // (first tile, count) per chunk
  std::vector<SymTile> tiles;
  std::vector<int32_t> csrc;
  int64_t stot = 0, ttot = 0;
  for (int32_t t = 0; t < nc; ++t) {
    if (rowblk[t].empty()) continue;
    const int32_t lt = rank[t];
    int64_t K = 0;
    for (int64_t b : rowblk[t]) {
      colstart[b] = (int32_t)K;
      K += rank[h->adm_col[b]];
    }
    if (K > INT32_MAX || (int64_t)csrc.size() + K > INT32_MAX) return fail(UHM_ENOTSUP, "coupling row too wide");
    const int32_t cs0 = (int32_t)csrc.size();
    for (int64_t b : rowblk[t])
      for (int32_t j = 0; j < rank[h->adm_col[b]]; ++j) csrc.push_back((int32_t)(rs_off[h->adm_col[b]] + j));
    for (int32_t r0 = 0; r0 < lt; r0 += kRowChunk) {
      const int32_t hh = std::min(kRowChunk, lt - r0);
      chunk_tp[t].push_back(ttot);
      const int32_t t0 = (int32_t)tiles.size();
      for (int64_t c0 = 0; c0 < K; c0 += kCoupCols) {
        const int32_t ncol = (int32_t)std::min<int64_t>(kCoupCols, K - c0);
        tiles.push_back({stot + c0 * hh, ttot + c0, cs0 + (int32_t)c0, hh, ncol, (int32_t)(rs_off[t] + r0)});
      }
      chunk_tiles[t].push_back({t0, (int32_t)tiles.size() - t0});
      stot += K * hh;
      ttot += K;
    }
  }
  if (tiles.size() > (size_t)INT32_MAX / kRowChunk) return fail(UHM_ENOTSUP, "too many coupling tiles");
  // result groups: every cluster with a basis, in row chunks; direct tiles of its own
  // stored blocks, then the transposed partials of the blocks stored on the mirror side
  std::vector<int64_t> grp_start, tsrc;
  std::vector<int32_t> grp_t0, grp_nt, grp_s0, grp_ns, yh_grp(nrs);
  for (int32_t c = 0; c < nc; ++c) {
    if (rank[c] < 1) continue;
    for (int32_t r0 = 0, ci = 0; r0 < rank[c]; r0 += kRowChunk, ++ci) {
      const int32_t hh = std::min(kRowChunk, rank[c] - r0);
      const int32_t g = (int32_t)grp_start.size();
      grp_start.push_back(rs_off[c] + r0);
      if (!rowblk[c].empty()) {
        grp_t0.push_back(chunk_tiles[c][ci].first);
        grp_nt.push_back(chunk_tiles[c][ci].second);
      } else {
        grp_t0.push_back(0);
        grp_nt.push_back(0);
      }
      if (tsrc.size() > (size_t)INT32_MAX) return fail(UHM_ENOTSUP, "transposed source table too large");
      grp_s0.push_back((int32_t)tsrc.size());
      for (int64_t b : colblk[c])
        for (int64_t base : chunk_tp[h->adm_row[b]]) tsrc.push_back(base + colstart[b] + r0);
      if (tsrc.size() - grp_s0.back() > (size_t)INT32_MAX) return fail(UHM_ENOTSUP, "transposed source table too large");
      grp_ns.push_back((int32_t)(tsrc.size() - grp_s0.back()));
      for (int32_t r = 0; r < hh; ++r) yh_grp[rs_off[c] + r0 + r] = g;
    }
  }
  // slack after the couplings, the backward panels and the column-source table: the
  // last 8-column group of a tile or panel range may read up to 7 columns past its end
  if (!tiles.empty()) csrc.insert(csrc.end(), 8, 0);
  if ((rc = op->S.alloc(stot + kSymSlack))) return rc;
  UHM_HIP(hipMemsetAsync(op->S.p + stot, 0, sizeof(cd) * kSymSlack, s));
  if (stot > 0) {
    Stager st;
    if ((rc = st.init(op->S.p, stot, s))) return rc;
    for (int32_t t = 0; t < nc && !st.err; ++t) {
      if (rowblk[t].empty()) continue;
      const int32_t lt = rank[t];
      for (int32_t r0 = 0; r0 < lt; r0 += kRowChunk) {
        const int32_t hh = std::min(kRowChunk, lt - r0);
        for (int64_t b : rowblk[t]) {
          const int32_t ls = rank[h->adm_col[b]];
          const cd* Sb = Sh + h->S_off[b];
          for (int32_t j = 0; j < ls; ++j) {
            cd* dst = st.span(hh);
            std::memcpy(static_cast<void*>(dst), Sb + (int64_t)j * lt + r0, sizeof(cd) * (size_t)hh);
          }
        }
      }
    }
    if ((rc = st.finish())) return rc;
  }

  // ---- backward panels: ancestor bases, diagonal dense blocks, then the stored
  // off-diagonal dense blocks (also applied transposed)
  std::vector<std::vector<int64_t>> dendiag(nc), denoff(nc);
  for (int64_t b = 0; b < h->nden; ++b)
    (h->den_row[b] == h->den_col[b] ? dendiag : denoff)[h->den_row[b]].push_back(b);
  std::vector<int64_t> bwd_off(nl), zoff(nl), td_off(nl);
  std::vector<int32_t> bwd_cols(nl), bwd_tcol(nl), leaf_n(nl);
  int64_t btot = 0, ztot = 0, tdtot = 0;
  for (int32_t i = 0; i < nl; ++i) {
    int64_t K = 0;
    for (int32_t a : T.anc[i]) {
      K += rank[a];
      for (int64_t b : dendiag[a]) K += h->size[h->den_col[b]];
    }
    const int64_t tc = K;
    for (int32_t a : T.anc[i])
      for (int64_t b : denoff[a]) K += h->size[h->den_col[b]];
    if (K > INT32_MAX) return fail(UHM_ENOTSUP, "backward panel too wide");
    leaf_n[i] = (int32_t)h->size[T.leaves[i]];
    bwd_cols[i] = (int32_t)K;
    bwd_tcol[i] = (int32_t)tc;
    bwd_off[i] = btot;
    zoff[i] = ztot;
    td_off[i] = tdtot;
    btot += K * leaf_n[i];
    ztot += K;
    tdtot += K - tc;
  }
  std::vector<int32_t> zmap(ztot);
  std::vector<std::vector<int64_t>> fin(nl);  // per output leaf: transposed partials to add
  if ((rc = op->B.alloc(btot + kSymSlack))) return rc;
  UHM_HIP(hipMemsetAsync(op->B.p + btot, 0, sizeof(cd) * kSymSlack, s));
  {
    Stager st;
    if ((rc = st.init(op->B.p, btot, s))) return rc;
    std::vector<PanelSeg> segs;
    for (int32_t i = 0; i < nl && !st.err; ++i) {
      const int32_t lf = T.leaves[i];
      segs.clear();
      int64_t z = zoff[i];
      auto dense = [&](int64_t b, int32_t a) {
        const int32_t sg = h->den_col[b];
        segs.push_back({D + h->D_off[b], h->size[a], h->off[lf] - h->off[a], (int32_t)h->size[sg], -1, nullptr});
        for (int64_t j = 0; j < h->size[sg]; ++j) zmap[z++] = (int32_t)(-1 - h->perm[h->off[sg] + j]);
      };
      for (int32_t a : T.anc[i])
        if (rank[a] > 0) {
          segs.push_back({U + h->U_off[a], h->size[a], h->off[lf] - h->off[a], rank[a], 0, nullptr});
          for (int32_t j = 0; j < rank[a]; ++j) zmap[z++] = (int32_t)(rs_off[a] + j);
        }
      for (int32_t a : T.anc[i])
        for (int64_t b : dendiag[a]) dense(b, a);
      for (int32_t a : T.anc[i])
        for (int64_t b : denoff[a]) {
          // column j of this block in leaf i's panel adds to row off[sg] + j; leaf mu of sg
          // reads its rows from td_off[i] + (panel column - tcol) + off[mu] - off[sg]
          const int32_t sg = h->den_col[b];
          const int64_t base = td_off[i] + (z - zoff[i]) - bwd_tcol[i];
          for (int32_t q = 0; q < T.leaf_cnt[sg]; ++q) {
            const int32_t mu = T.leaf_first[sg] + q;
            fin[mu].push_back(base + h->off[T.leaves[mu]] - h->off[sg]);
          }
          dense(b, a);
        }
      if ((rc = stage_backward_leaf(st, segs, (int32_t)h->size[lf]))) return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  std::vector<int32_t> fin_off(nl), fin_cnt(nl);
  std::vector<int64_t> fsrc;
  for (int32_t i = 0; i < nl; ++i) {
    if (fsrc.size() + fin[i].size() > (size_t)INT32_MAX) return fail(UHM_ENOTSUP, "finish table too large");
    fin_off[i] = (int32_t)fsrc.size();
    fin_cnt[i] = (int32_t)fin[i].size();
    fsrc.insert(fsrc.end(), fin[i].begin(), fin[i].end());
  }
  {
    LayoutView L{h->n, nl, FL.ftot, FL.ptot, btot, ztot, nrs, nrs, &leaf_n, &FL.fwd_off, &FL.fwd_cols, &FL.poff,
                 &FL.segs, &bwd_off, &bwd_cols, &zoff, &zmap};
    if ((rc = check_layout(L))) return rc;
    if ((rc = check_sym(tiles, stot, ttot, csrc, nrs, grp_start, grp_t0, grp_nt, grp_s0, grp_ns, tsrc, leaf_n,
                        bwd_cols, bwd_tcol, td_off, tdtot, fin_off, fin_cnt, fsrc)))
      return rc;
  }
  if ((rc = op->stiles.upload(tiles, s)) || (rc = op->csrc.upload(csrc, s)) || (rc = op->yh_grp.upload(yh_grp, s)) ||
      (rc = op->grp_start.upload(grp_start, s)) || (rc = op->grp_t0.upload(grp_t0, s)) ||
      (rc = op->grp_nt.upload(grp_nt, s)) || (rc = op->grp_s0.upload(grp_s0, s)) ||
      (rc = op->grp_ns.upload(grp_ns, s)) || (rc = op->tsrc.upload(tsrc, s)) ||
      (rc = op->bwd_off.upload(bwd_off, s)) || (rc = op->bwd_cols.upload(bwd_cols, s)) ||
      (rc = op->bwd_tcol.upload(bwd_tcol, s)) || (rc = op->td_off.upload(td_off, s)) ||
      (rc = op->zoff.upload(zoff, s)) || (rc = op->zmap.upload(zmap, s)) || (rc = op->fin_off.upload(fin_off, s)) ||
      (rc = op->fin_cnt.upload(fin_cnt, s)) || (rc = op->fsrc.upload(fsrc, s)))
    return rc;
  UHM_HIP(hipStreamSynchronize(s));
  op->sym = true;
  op->nctiles = (int32_t)tiles.size();
  op->nyh = nrs;
  op->ttot = ttot;
  op->tdtot = tdtot;

  uhm_op_info& I = op->info;
  I.n = h->n;
  I.kind = 0;
  I.storage = UHM_C128_SYM;
  I.nleaves = nl;
  I.elem_bytes = 16;
  I.nadm = h->nadm;
  I.nden = h->nden;
  I.elems_forward = I.elems_backward = 0;
  for (int32_t c = 0; c < nc; ++c) I.elems_forward += h->size[c] * rank[c];
  I.elems_backward = I.elems_forward;
  I.elems_coupling = stot;
  I.elems_near = 0;
  for (int64_t b = 0; b < h->nden; ++b) I.elems_near += h->size[h->den_row[b]] * h->size[h->den_col[b]];
  I.rank_space = nrs;
  I.partial_coupling = ttot;
  I.partial_near = tdtot;
  I.device_bytes = (int64_t)(op->F.bytes() + op->S.bytes() + op->B.bytes() + op->zmap.bytes() + op->perm.bytes() +
                             op->stiles.bytes() + op->csrc.bytes() + op->tsrc.bytes() + op->fsrc.bytes() +
                             op->out_seg.bytes() + op->yh_grp.bytes());
  return UHM_OK;
}

}  // namespace

namespace uhm_detail {
int grow_workspace_fp64(uhm_op* op) { return grow_workspace(op); }
}  // namespace uhm_detail

extern "C" {

int uhm_version(void) { return 1; }

const char* uhm_strerror(int code) {
  switch (code) {
    case UHM_OK: return "success";
    case UHM_EINVAL: return "invalid argument";
    case UHM_ENOMEM: return "out of memory";
    case UHM_EHIP: return "HIP runtime error";
    case UHM_ENOCONV: return "iteration limit reached without convergence";
    case UHM_ENOTSUP: return "not supported by the library";
    default: return "unknown error";
  }
}

const char* uhm_last_error(void) { return g_err.c_str(); }

int uhm_upload(const uhm_host_operator* h, uhm_storage storage, void* hip_stream, uhm_op** out) {
  if (!h || !out) return fail(UHM_EINVAL, "null argument");
  *out = nullptr;
  if (storage != UHM_C128 && storage != UHM_C64 && storage != UHM_BF16PAIR && storage != UHM_C128_MULTI &&
      storage != UHM_C128_SYM && storage != UHM_C128_FACTORED && storage != UHM_C64_FACTORED &&
      storage != UHM_BF16PAIR_FACTORED && storage != UHM_C128_MULTI_FACTORED && !is_stream(storage))
    return fail(UHM_EINVAL, "unknown storage precision");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  TreeInfo T;
  int rc = check_tree(h->n, h->perm, h->nclusters, h->off, h->size, h->parent, T);
  if (rc) return rc;
  const int32_t nc = h->nclusters;
  if (storage == UHM_C128_SYM) {
    std::unique_ptr<uhm_op> op(new (std::nothrow) uhm_op);
    if (!op) return fail(UHM_ENOMEM, "host allocation");
    op->kind = 0;
    op->storage = storage;
    if ((rc = common_tree_upload(op.get(), T, h->perm, h->off, h->size, s))) return rc;
    if ((rc = upload_sym(h, s, T, op.get()))) return rc;
    *out = op.release();
    return UHM_OK;
  }
  if (!h->rank_row || !h->rank_col || !h->U_off || !h->V_off) return fail(UHM_EINVAL, "null basis arrays");
  if ((h->nadm > 0 && (!h->adm_row || !h->adm_col || !h->S_off || !h->S)) ||
      (h->nden > 0 && (!h->den_row || !h->den_col || !h->D_off || !h->D)) || h->nadm < 0 || h->nden < 0)
    return fail(UHM_EINVAL, "null block arrays");
  for (int32_t c = 0; c < nc; ++c) {
    if (h->rank_row[c] < 0 || h->rank_col[c] < 0 || h->rank_row[c] > h->size[c] || h->rank_col[c] > h->size[c])
      return fail(UHM_EINVAL, "cluster rank out of range");
    if (h->rank_row[c] > 0 && (!h->U || !in_bounds(h->U_off[c], h->size[c] * h->rank_row[c], h->U_len)))
      return fail(UHM_EINVAL, "U_off out of bounds");
    if (h->rank_col[c] > 0 && (!h->V || !in_bounds(h->V_off[c], h->size[c] * h->rank_col[c], h->V_len)))
      return fail(UHM_EINVAL, "V_off out of bounds");
  }
  for (int64_t b = 0; b < h->nadm; ++b) {
    const int32_t t = h->adm_row[b], sg = h->adm_col[b];
    if (t < 0 || t >= nc || sg < 0 || sg >= nc) return fail(UHM_EINVAL, "admissible block cluster out of range");
    if (h->rank_row[t] < 1 || h->rank_col[sg] < 1) return fail(UHM_EINVAL, "admissible block without bases");
    if (!in_bounds(h->S_off[b], (int64_t)h->rank_row[t] * h->rank_col[sg], h->S_len))
      return fail(UHM_EINVAL, "S_off out of bounds");
  }
  for (int64_t b = 0; b < h->nden; ++b) {
    const int32_t t = h->den_row[b], sg = h->den_col[b];
    if (t < 0 || t >= nc || sg < 0 || sg >= nc) return fail(UHM_EINVAL, "dense block cluster out of range");
    if (!in_bounds(h->D_off[b], h->size[t] * h->size[sg], h->D_len)) return fail(UHM_EINVAL, "D_off out of bounds");
  }
  // factored couplings: which blocks take the two-step form (fewer stored elements)
  const bool factored = storage == UHM_C128_FACTORED || storage == UHM_C64_FACTORED ||
                        storage == UHM_BF16PAIR_FACTORED || storage == UHM_C128_MULTI_FACTORED;
  std::vector<char> fac(h->nadm, 0);
  if (factored) {
    if (h->nadm > 0 && (!h->adm_rank || !h->SX_off || !h->SY_off || !h->SX || !h->SY))
      return fail(UHM_EINVAL, "factored storage needs adm_rank, SX and SY");
    for (int64_t b = 0; b < h->nadm; ++b) {
      const int64_t lt = h->rank_row[h->adm_row[b]], ls = h->rank_col[h->adm_col[b]], k = h->adm_rank[b];
      if (k < 1 || !in_bounds(h->SX_off[b], lt * k, h->SX_len) || !in_bounds(h->SY_off[b], ls * k, h->SY_len))
        return fail(UHM_EINVAL, "factored coupling out of bounds");
      fac[b] = k * (lt + ls) < lt * ls;
    }
  }
  std::unique_ptr<uhm_op> op(new (std::nothrow) uhm_op);
  if (!op) return fail(UHM_ENOMEM, "host allocation");
  op->kind = 0;
  op->storage = storage;
  if ((rc = common_tree_upload(op.get(), T, h->perm, h->off, h->size, s))) return rc;
  if (storage != UHM_C128 && storage != UHM_C128_FACTORED && !is_stream(storage)) {
    if ((rc = lowp_upload(h, storage, s, T, op.get()))) return rc;
    *out = op.release();
    return UHM_OK;
  }
  const int32_t nl = op->nleaves;
  const cd* U = reinterpret_cast<const cd*>(h->U);
  const cd* V = reinterpret_cast<const cd*>(h->V);
  const cd* Sh = reinterpret_cast<const cd*>(h->S);
  const cd* D = reinterpret_cast<const cd*>(h->D);

  // ---- rank-space vectors: u_sigma at xh_off[sigma], u_tau at yh_off[tau]
  std::vector<int64_t> xh_off(nc, -1), yh_off(nc, -1);
  int64_t nxh = 0, nyh = 0;
  for (int32_t c = 0; c < nc; ++c) {
    if (h->rank_col[c] > 0) { xh_off[c] = nxh; nxh += h->rank_col[c]; }
    if (h->rank_row[c] > 0) { yh_off[c] = nyh; nyh += h->rank_row[c]; }
  }
  if (nxh > INT32_MAX || nyh > INT32_MAX) return fail(UHM_ENOTSUP, "rank space too large");

  // ---- forward panels
  FwdLayout FL;
  if ((rc = build_forward(op.get(), T, h->off, h->size, h->rank_col, V, h->V_off, false, xh_off, nxh, s, FL))) return rc;

  // ---- factored couplings, first step: t_b = S_{Y,b}^* u_sigma, stored in the coupling source
  // vector after u, block by block within each column cluster
  std::vector<int64_t> t_off(h->nadm, -1);
  std::vector<std::vector<int64_t>> colfac(nc);
  for (int64_t b = 0; b < h->nadm; ++b)
    if (fac[b]) colfac[h->adm_col[b]].push_back(b);
  int64_t nsrc = nxh;
  for (int32_t c = 0; c < nc; ++c)
    for (int64_t b : colfac[c]) {
      t_off[b] = nsrc;
      nsrc += h->adm_rank[b];
    }
  if (nsrc > INT32_MAX) return fail(UHM_ENOTSUP, "coupling source vector too long");
  std::vector<FacTile> ftl;
  int64_t fytot = 0;
  for (int32_t c = 0; c < nc; ++c) {
    int64_t Kf = 0;
    for (int64_t b : colfac[c]) Kf += h->adm_rank[b];
    for (int64_t c0 = 0; c0 < Kf; c0 += kTile) {
      const int32_t wj = (int32_t)std::min<int64_t>(kTile, Kf - c0);
      ftl.push_back({fytot, h->rank_col[c], wj, (int32_t)xh_off[c], (int32_t)(t_off[colfac[c][0]] + c0)});
      fytot += (int64_t)wj * h->rank_col[c];
    }
  }
  if (ftl.size() > (size_t)INT32_MAX) return fail(UHM_ENOTSUP, "too many factor tiles");
  if ((rc = op->FY.alloc(fytot))) return rc;
  if (fytot > 0) {
    const cd* SY = reinterpret_cast<const cd*>(h->SY);
    Stager st;
    if ((rc = st.init(op->FY.p, fytot, s))) return rc;
    std::vector<const cd*> colp;
    for (int32_t c = 0; c < nc && !st.err; ++c) {
      if (colfac[c].empty()) continue;
      const int32_t ls = h->rank_col[c];
      colp.clear();  // start of every panel column, in the order of the t_b
      for (int64_t b : colfac[c])
        for (int32_t j = 0; j < h->adm_rank[b]; ++j) colp.push_back(SY + h->SY_off[b] + (int64_t)j * ls);
      for (size_t c0 = 0; c0 < colp.size(); c0 += kTile) {
        const int32_t wj = (int32_t)std::min<size_t>(kTile, colp.size() - c0);
        cd* tile = st.span((int64_t)wj * ls);
        for (int32_t r = 0; r < ls; ++r)
          for (int32_t q = 0; q < wj; ++q) tile[(int64_t)r * wj + q] = colp[c0 + q][r];
      }
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = op->factiles.upload(ftl, s))) return rc;
  op->nfactiles = (int32_t)ftl.size();
  op->nsrc = nsrc;

  // ---- couplings, grouped by row cluster, in row chunks: [S_b1 S_b2 ...] with a factored
  // block's S_{X,b} in place of its S_b
  std::vector<std::vector<int64_t>> rowblk(nc);
  for (int64_t b = 0; b < h->nadm; ++b) rowblk[h->adm_row[b]].push_back(b);
  auto width = [&](int64_t b) { return fac[b] ? h->adm_rank[b] : h->rank_col[h->adm_col[b]]; };
  std::vector<CoupTile> tiles;
  std::vector<int2> cblk;
  std::vector<int32_t> grp_t0, grp_nt, yh_grp(nyh);
  std::vector<int64_t> grp_start;
  int64_t stot = 0;
  for (int32_t t = 0; t < nc; ++t) {
    if (rowblk[t].empty()) continue;
    std::sort(rowblk[t].begin(), rowblk[t].end());
    const int32_t lt = h->rank_row[t];
    int64_t K = 0;
    for (int64_t b : rowblk[t]) K += width(b);
    const int32_t blk0 = (int32_t)cblk.size();
    for (int64_t b : rowblk[t])
      cblk.push_back(make_int2(width(b), (int32_t)(fac[b] ? t_off[b] : xh_off[h->adm_col[b]])));
    for (int32_t r0 = 0; r0 < lt; r0 += kRowChunk) {
      const int32_t hh = std::min(kRowChunk, lt - r0);
      const int32_t g = (int32_t)grp_start.size();
      grp_start.push_back(yh_off[t] + r0);
      grp_t0.push_back((int32_t)tiles.size());
      for (int32_t r = 0; r < hh; ++r) yh_grp[yh_off[t] + r0 + r] = g;
      int32_t bi = 0, bj = 0;
      for (int64_t c0 = 0; c0 < K; c0 += kCoupCols) {
        const int32_t nc_ = (int32_t)std::min<int64_t>(kCoupCols, K - c0);
        tiles.push_back({stot + c0 * hh, hh, nc_, blk0 + bi, bj});
        // advance the block cursor by nc_ columns
        int32_t left = nc_;
        while (left > 0) {
          const int32_t len = cblk[blk0 + bi].x;
          const int32_t take = std::min(len - bj, left);
          left -= take;
          bj += take;
          if (bj == len) { ++bi; bj = 0; }
        }
      }
      grp_nt.push_back((int32_t)tiles.size() - grp_t0.back());
      stot += K * hh;
    }
  }
  if (tiles.size() > (size_t)INT32_MAX / kRowChunk) return fail(UHM_ENOTSUP, "too many coupling tiles");
  if ((rc = op->S.alloc(stot))) return rc;
  if (stot > 0) {
    Stager st;
    if ((rc = st.init(op->S.p, stot, s))) return rc;
    for (int32_t t = 0; t < nc && !st.err; ++t) {
      if (rowblk[t].empty()) continue;
      const int32_t lt = h->rank_row[t];
      for (int32_t r0 = 0; r0 < lt; r0 += kRowChunk) {
        const int32_t hh = std::min(kRowChunk, lt - r0);
        for (int64_t b : rowblk[t]) {
          const int32_t ls = (int32_t)width(b);
          const cd* Sb = fac[b] ? reinterpret_cast<const cd*>(h->SX) + h->SX_off[b] : Sh + h->S_off[b];
          for (int32_t j = 0; j < ls; ++j) {
            cd* dst = st.span(hh);
            std::memcpy(static_cast<void*>(dst), Sb + (int64_t)j * lt + r0, sizeof(cd) * (size_t)hh);
          }
        }
      }
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = op->ctiles.upload(tiles, s)) || (rc = op->cblk.upload(cblk, s)) || (rc = op->yh_grp.upload(yh_grp, s)) ||
      (rc = op->grp_start.upload(grp_start, s)) || (rc = op->grp_t0.upload(grp_t0, s)) ||
      (rc = op->grp_nt.upload(grp_nt, s)))
    return rc;
  op->nctiles = (int32_t)tiles.size();
  op->nyh = nyh;

  // ---- backward panels: ancestor bases, then dense blocks of the leaf's rows
  std::vector<std::vector<int64_t>> denrow(nc);
  for (int64_t b = 0; b < h->nden; ++b) denrow[h->den_row[b]].push_back(b);
  std::vector<int64_t> bwd_off(nl), zoff(nl);
  std::vector<int32_t> bwd_cols(nl);
  int64_t btot = 0, ztot = 0;
  for (int32_t i = 0; i < nl; ++i) {
    int64_t K = 0;
    for (int32_t a : T.anc[i]) {
      K += h->rank_row[a];
      for (int64_t b : denrow[a]) K += h->size[h->den_col[b]];
    }
    if (K > INT32_MAX) return fail(UHM_ENOTSUP, "backward panel too wide");
    bwd_cols[i] = (int32_t)K;
    bwd_off[i] = btot;
    zoff[i] = ztot;
    btot += K * h->size[T.leaves[i]];
    ztot += K;
  }
  std::vector<int32_t> zmap(ztot);
  if ((rc = op->B.alloc(btot))) return rc;
  {
    Stager st;
    if ((rc = st.init(op->B.p, btot, s))) return rc;
    std::vector<PanelSeg> segs;
    for (int32_t i = 0; i < nl && !st.err; ++i) {
      const int32_t lf = T.leaves[i];
      segs.clear();
      int64_t z = zoff[i];
      for (int32_t a : T.anc[i])
        if (h->rank_row[a] > 0) {
          segs.push_back({U + h->U_off[a], h->size[a], h->off[lf] - h->off[a], h->rank_row[a], 0, nullptr});
          for (int32_t j = 0; j < h->rank_row[a]; ++j) zmap[z++] = (int32_t)(yh_off[a] + j);
        }
      for (int32_t a : T.anc[i])
        for (int64_t b : denrow[a]) {
          const int32_t sg = h->den_col[b];
          segs.push_back({D + h->D_off[b], h->size[a], h->off[lf] - h->off[a], (int32_t)h->size[sg], -1, nullptr});
          for (int64_t j = 0; j < h->size[sg]; ++j) zmap[z++] = (int32_t)(-1 - h->perm[h->off[sg] + j]);
        }
      if ((rc = stage_backward_leaf(st, segs, (int32_t)h->size[lf]))) return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = op->bwd_off.upload(bwd_off, s)) || (rc = op->bwd_cols.upload(bwd_cols, s)) ||
      (rc = op->zoff.upload(zoff, s)) || (rc = op->zmap.upload(zmap, s)))
    return rc;
  UHM_HIP(hipStreamSynchronize(s));
  {
    std::vector<int32_t> leaf_n(nl);
    for (int32_t i = 0; i < nl; ++i) leaf_n[i] = (int32_t)h->size[T.leaves[i]];
    LayoutView L{h->n, nl, FL.ftot, FL.ptot, btot, ztot, nyh, nxh, &leaf_n, &FL.fwd_off, &FL.fwd_cols, &FL.poff, &FL.segs,
                 &bwd_off, &bwd_cols, &zoff, &zmap};
    if ((rc = check_layout(L))) return rc;
    if ((rc = check_coupling(tiles, cblk, stot, nsrc, grp_t0, grp_nt, grp_start, nyh))) return rc;
    for (const FacTile& F : ftl)
      if (F.rows < 1 || F.wj < 1 || F.wj > kTile || F.f_base < 0 || F.f_base + (int64_t)F.rows * F.wj > fytot ||
          F.x_row < 0 || (int64_t)F.x_row + F.rows > nxh || F.t_out < nxh || (int64_t)F.t_out + F.wj > nsrc)
        return fail(UHM_EINVAL, "layout: factor tile");
  }

  uhm_op_info& I = op->info;
  I.n = h->n;
  I.kind = 0;
  I.storage = storage;
  I.nleaves = nl;
  I.elem_bytes = 16;
  I.nadm = h->nadm;
  I.nden = h->nden;
  I.elems_forward = I.elems_backward = 0;
  for (int32_t c = 0; c < nc; ++c) {
    I.elems_forward += h->size[c] * h->rank_col[c];
    I.elems_backward += h->size[c] * h->rank_row[c];
  }
  I.elems_coupling = stot;
  I.elems_coupling_in = fytot;
  I.elems_near = 0;
  for (int64_t b = 0; b < h->nden; ++b) I.elems_near += h->size[h->den_row[b]] * h->size[h->den_col[b]];
  I.rank_space = nxh;
  if (is_stream(storage)) {
    // the complex128 panels become the storage element
    if ((rc = stream_compact(op.get(), s))) return rc;
    I.elem_bytes = storage == UHM_C64_STREAM ? 8 : 4;
  }
  I.device_bytes = (int64_t)(op->F.bytes() + op->S.bytes() + op->B.bytes() + op->Fs.bytes() + op->Ss.bytes() +
                             op->Bs.bytes() + op->zmap.bytes() + op->perm.bytes() + op->ctiles.bytes() +
                             op->cblk.bytes() + op->out_seg.bytes() + op->yh_grp.bytes() + op->FY.bytes() +
                             op->factiles.bytes());
  *out = op.release();
  return UHM_OK;
}

int uhm_upload_h(const uhm_host_hmatrix* h, uhm_storage storage, void* hip_stream, uhm_op** out) {
  if (!h || !out) return fail(UHM_EINVAL, "null argument");
  *out = nullptr;
  if (storage != UHM_C128) return fail(UHM_ENOTSUP, "the H-matrix form is stored in complex128 only");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  TreeInfo T;
  int rc = check_tree(h->n, h->perm, h->nclusters, h->off, h->size, h->parent, T);
  if (rc) return rc;
  const int32_t nc = h->nclusters;
  if ((h->nadm > 0 && (!h->adm_row || !h->adm_col || !h->adm_rank || !h->X_off || !h->Y_off || !h->X || !h->Y)) ||
      (h->nden > 0 && (!h->den_row || !h->den_col || !h->D_off || !h->D)) || h->nadm < 0 || h->nden < 0)
    return fail(UHM_EINVAL, "null block arrays");
  for (int64_t b = 0; b < h->nadm; ++b) {
    const int32_t t = h->adm_row[b], sg = h->adm_col[b];
    if (t < 0 || t >= nc || sg < 0 || sg >= nc) return fail(UHM_EINVAL, "admissible block cluster out of range");
    const int32_t k = h->adm_rank[b];
    if (k < 1 || k > std::min(h->size[t], h->size[sg])) return fail(UHM_EINVAL, "block rank out of range");
    if (!in_bounds(h->X_off[b], h->size[t] * k, h->X_len) || !in_bounds(h->Y_off[b], h->size[sg] * k, h->Y_len))
      return fail(UHM_EINVAL, "X_off/Y_off out of bounds");
  }
  for (int64_t b = 0; b < h->nden; ++b) {
    const int32_t t = h->den_row[b], sg = h->den_col[b];
    if (t < 0 || t >= nc || sg < 0 || sg >= nc) return fail(UHM_EINVAL, "dense block cluster out of range");
    if (!in_bounds(h->D_off[b], h->size[t] * h->size[sg], h->D_len)) return fail(UHM_EINVAL, "D_off out of bounds");
  }
  std::unique_ptr<uhm_op> op(new (std::nothrow) uhm_op);
  if (!op) return fail(UHM_ENOMEM, "host allocation");
  op->kind = 1;
  op->storage = storage;
  if ((rc = common_tree_upload(op.get(), T, h->perm, h->off, h->size, s))) return rc;
  const int32_t nl = op->nleaves;
  const cd* X = reinterpret_cast<const cd*>(h->X);
  const cd* Y = reinterpret_cast<const cd*>(h->Y);
  const cd* D = reinterpret_cast<const cd*>(h->D);
  std::vector<std::vector<int64_t>> colblk(nc), rowblk(nc), denrow(nc);
  for (int64_t b = 0; b < h->nadm; ++b) {
    colblk[h->adm_col[b]].push_back(b);
    rowblk[h->adm_row[b]].push_back(b);
  }
  for (int64_t b = 0; b < h->nden; ++b) denrow[h->den_row[b]].push_back(b);
  // t_b = Y_b^* v|_sigma at t_off[b]
  std::vector<int64_t> t_off(h->nadm);
  int64_t nt = 0;
  for (int64_t b = 0; b < h->nadm; ++b) { t_off[b] = nt; nt += h->adm_rank[b]; }
  if (nt > INT32_MAX) return fail(UHM_ENOTSUP, "rank space too large");

  // ---- forward panels from Y_b, one segment per block of each ancestor column cluster
  std::vector<int64_t> fwd_off(nl), poff(nl);
  std::vector<int32_t> fwd_cols(nl);
  std::vector<int32_t> bcol(h->nadm, -1);
  int64_t ftot = 0, ptot = 0;
  for (int32_t i = 0; i < nl; ++i) {
    int64_t C = 0;
    for (int32_t a : T.anc[i])
      for (int64_t b : colblk[a]) {
        if (bcol[b] < 0) bcol[b] = (int32_t)C;
        C += h->adm_rank[b];
      }
    if (C > INT32_MAX) return fail(UHM_ENOTSUP, "forward panel too wide");
    fwd_cols[i] = (int32_t)C;
    fwd_off[i] = ftot;
    poff[i] = ptot;
    ftot += C * h->size[T.leaves[i]];
    ptot += C;
  }
  if ((rc = op->F.alloc(ftot))) return rc;
  {
    Stager st;
    if ((rc = st.init(op->F.p, ftot, s))) return rc;
    std::vector<PanelSeg> segs;
    for (int32_t i = 0; i < nl && !st.err; ++i) {
      const int32_t lf = T.leaves[i];
      segs.clear();
      for (int32_t a : T.anc[i])
        for (int64_t b : colblk[a])
          segs.push_back({Y + h->Y_off[b], h->size[a], h->off[lf] - h->off[a], h->adm_rank[b], -1, nullptr});
      if ((rc = stage_forward_leaf(st, segs, fwd_cols[i], (int32_t)h->size[lf]))) return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = op->fwd_off.upload(fwd_off, s)) || (rc = op->fwd_cols.upload(fwd_cols, s)) ||
      (rc = upload_fwd_tiles(op.get(), fwd_cols, s)) ||
      (rc = op->poff.upload(poff, s)))
    return rc;
  op->p_len = ptot;
  {
    std::vector<SegDesc> segs;
    for (int64_t b = 0; b < h->nadm; ++b) {
      const int32_t sg = h->adm_col[b];
      segs.push_back({t_off[b], h->adm_rank[b], T.leaf_first[sg], T.leaf_cnt[sg], bcol[b]});
    }
    if ((rc = upload_segments(op.get(), segs, nt, s))) return rc;
  }

  // ---- backward panels from X_b, then dense blocks
  std::vector<int64_t> bwd_off(nl), zoff(nl);
  std::vector<int32_t> bwd_cols(nl);
  int64_t btot = 0, ztot = 0;
  for (int32_t i = 0; i < nl; ++i) {
    int64_t K = 0;
    for (int32_t a : T.anc[i]) {
      for (int64_t b : rowblk[a]) K += h->adm_rank[b];
      for (int64_t b : denrow[a]) K += h->size[h->den_col[b]];
    }
    if (K > INT32_MAX) return fail(UHM_ENOTSUP, "backward panel too wide");
    bwd_cols[i] = (int32_t)K;
    bwd_off[i] = btot;
    zoff[i] = ztot;
    btot += K * h->size[T.leaves[i]];
    ztot += K;
  }
  std::vector<int32_t> zmap(ztot);
  if ((rc = op->B.alloc(btot))) return rc;
  {
    Stager st;
    if ((rc = st.init(op->B.p, btot, s))) return rc;
    std::vector<PanelSeg> segs;
    for (int32_t i = 0; i < nl && !st.err; ++i) {
      const int32_t lf = T.leaves[i];
      segs.clear();
      int64_t z = zoff[i];
      for (int32_t a : T.anc[i])
        for (int64_t b : rowblk[a]) {
          segs.push_back({X + h->X_off[b], h->size[a], h->off[lf] - h->off[a], h->adm_rank[b], 0, nullptr});
          for (int32_t j = 0; j < h->adm_rank[b]; ++j) zmap[z++] = (int32_t)(t_off[b] + j);
        }
      for (int32_t a : T.anc[i])
        for (int64_t b : denrow[a]) {
          const int32_t sg = h->den_col[b];
          segs.push_back({D + h->D_off[b], h->size[a], h->off[lf] - h->off[a], (int32_t)h->size[sg], -1, nullptr});
          for (int64_t j = 0; j < h->size[sg]; ++j) zmap[z++] = (int32_t)(-1 - h->perm[h->off[sg] + j]);
        }
      if ((rc = stage_backward_leaf(st, segs, (int32_t)h->size[lf]))) return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = op->bwd_off.upload(bwd_off, s)) || (rc = op->bwd_cols.upload(bwd_cols, s)) ||
      (rc = op->zoff.upload(zoff, s)) || (rc = op->zmap.upload(zmap, s)))
    return rc;
  UHM_HIP(hipStreamSynchronize(s));
  {
    std::vector<int32_t> leaf_n(nl);
    for (int32_t i = 0; i < nl; ++i) leaf_n[i] = (int32_t)h->size[T.leaves[i]];
    std::vector<SegDesc> segs;
    for (int64_t b = 0; b < h->nadm; ++b) {
      const int32_t sg = h->adm_col[b];
      segs.push_back({t_off[b], h->adm_rank[b], T.leaf_first[sg], T.leaf_cnt[sg], bcol[b]});
    }
    LayoutView L{h->n, nl, ftot, ptot, btot, ztot, nt, nt, &leaf_n, &fwd_off, &fwd_cols, &poff, &segs,
                 &bwd_off, &bwd_cols, &zoff, &zmap};
    if ((rc = check_layout(L))) return rc;
  }

  uhm_op_info& I = op->info;
  I.n = h->n;
  I.kind = 1;
  I.storage = storage;
  I.nleaves = nl;
  I.elem_bytes = 16;
  I.nadm = h->nadm;
  I.nden = h->nden;
  I.elems_forward = I.elems_backward = 0;
  for (int64_t b = 0; b < h->nadm; ++b) {
    I.elems_forward += h->size[h->adm_col[b]] * h->adm_rank[b];
    I.elems_backward += h->size[h->adm_row[b]] * h->adm_rank[b];
  }
  I.elems_coupling = 0;
  I.elems_near = 0;
  for (int64_t b = 0; b < h->nden; ++b) I.elems_near += h->size[h->den_row[b]] * h->size[h->den_col[b]];
  I.rank_space = nt;
  I.device_bytes = (int64_t)(op->F.bytes() + op->B.bytes() + op->zmap.bytes() + op->perm.bytes() + op->out_seg.bytes());
  *out = op.release();
  return UHM_OK;
}

}  // extern "C"

namespace {

// Scratch of the complex128 single-RHS product: per-leaf forward partials, the coupling
// source vector, coupling partials, the rank-space result, and (symmetric storage) the
// transposed coupling and near-field partials.  Every entry a kernel reads is written
// earlier in the same product, so the contents at entry do not matter.
struct Fp64Ws {
  cd *p, *xh, *part, *yh, *tpart, *td;
};

// Element counts of the six scratch areas, in the order of Fp64Ws.
void fp64_ws_counts(const uhm_op* op, int64_t cnt[6]) {
  cnt[0] = op->p_len;
  cnt[1] = std::max(op->nxh, op->nsrc);
  cnt[2] = op->kind == 0 ? (int64_t)op->nctiles * kRowChunk : 0;
  cnt[3] = op->kind == 0 ? op->nyh : 0;
  cnt[4] = op->sym ? op->ttot : 0;
  cnt[5] = op->sym ? op->tdtot : 0;
}

// Offsets of the six areas in one scratch array, each on a 256-byte boundary (16
// complex128 elements); returns the total element count.
int64_t fp64_ws_layout(const uhm_op* op, int64_t off[6]) {
  int64_t cnt[6], tot = 0;
  fp64_ws_counts(op, cnt);
  for (int k = 0; k < 6; ++k) {
    off[k] = tot;
    tot += (cnt[k] + 15) / 16 * 16;
  }
  return tot;
}

int check_vectors(const uhm_op* op, const void* X, int64_t ldx, const void* Y, int64_t ldy, int32_t nrhs) {
  if (!X || !Y) return fail(UHM_EINVAL, "null vector pointer");
  if (ldx < op->n || ldy < op->n) return fail(UHM_EINVAL, "leading dimension smaller than n");
  const char* xb = static_cast<const char*>(X);
  const char* yb = static_cast<const char*>(Y);
  const size_t es = is_c128(op->storage) ? sizeof(cd) : sizeof(float2);
  if (xb < yb + (size_t)((nrhs - 1) * ldy + op->n) * es && yb < xb + (size_t)((nrhs - 1) * ldx + op->n) * es)
    return fail(UHM_EINVAL, "X and Y overlap");
  return UHM_OK;
}

int matvec_fp64(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, hipStream_t s,
                const Fp64Ws& w);

// File-scope scratch of uhm_matvec_noalloc, one copy per GPU.  Host code uses the
// device address that hipGetSymbolAddress returns for the current device (g_scratch_dev),
// never the array's name, which is a host-side stand-in.
constexpr int64_t kNoallocScratchBytes = int64_t(512) << 20;
__device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_address(void** out) {
  int dev = -1;
  UHM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(UHM_ENOTSUP, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    UHM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(UHM_EHIP, "hipGetSymbolAddress returned a null scratch address");
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return UHM_OK;
}

}  // namespace

extern "C" {

int uhm_matvec(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, void* hip_stream) {
  if (!op) return fail(UHM_EINVAL, "null operator");
  if (nrhs < 0) return fail(UHM_EINVAL, "nrhs < 0");
  if (nrhs == 0) return UHM_OK;
  int rc = check_vectors(op, X, ldx, Y, ldy, nrhs);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (op->lp) return lowp_matvec(op, X, ldx, Y, ldy, nrhs, s);
  if (is_stream(op->storage)) return stream_matvec(op, X, ldx, Y, ldy, nrhs, s);
  if ((rc = grow_workspace(op))) return rc;
  const Fp64Ws w{op->ws_p.p, op->ws_xh.p, op->ws_part.p, op->ws_yh.p, op->ws_tpart.p, op->ws_td.p};
  return matvec_fp64(op, X, ldx, Y, ldy, nrhs, s, w);
}

int uhm_matvec_noalloc(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs,
                       void* hip_stream) {
  if (!op) return fail(UHM_EINVAL, "null operator");
  if (nrhs < 0) return fail(UHM_EINVAL, "nrhs < 0");
  if (op->lp || !is_c128(op->storage))
    return fail(UHM_ENOTSUP, "uhm_matvec_noalloc takes the complex128 single-RHS storage forms only");
  if (nrhs == 0) return UHM_OK;
  int rc = check_vectors(op, X, ldx, Y, ldy, nrhs);
  if (rc) return rc;
  int64_t off[6];
  const int64_t tot = fp64_ws_layout(op, off);
  if (tot * (int64_t)sizeof(cd) > kNoallocScratchBytes)
    return fail(UHM_EINVAL, "operator needs " + std::to_string(tot * (int64_t)sizeof(cd)) +
                                " B of product scratch, more than the " + std::to_string(kNoallocScratchBytes) +
                                " B that uhm_matvec_noalloc holds");
  void* base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  cd* b = static_cast<cd*>(base);
  const Fp64Ws w{b + off[0], b + off[1], b + off[2], b + off[3], b + off[4], b + off[5]};
  return matvec_fp64(op, X, ldx, Y, ldy, nrhs, static_cast<hipStream_t>(hip_stream), w);
}

}  // extern "C"

namespace {

int matvec_fp64(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, hipStream_t s,
                const Fp64Ws& w) {
  const int nl = op->nleaves;
  for (int32_t r = 0; r < nrhs; ++r) {
    const cd* x = static_cast<const cd*>(X) + (int64_t)r * ldx;
    cd* y = static_cast<cd*>(Y) + (int64_t)r * ldy;
    if (op->nxh > 0) {
      {
        ScopedTiming tm(op, s, K_FORWARD);
        hipLaunchKernelGGL(op->kind == 0 ? k_forward_tiles<0> : k_forward_tiles<1>,
                           dim3((unsigned)((op->nftiles + kFwdWaves - 1) / kFwdWaves)), dim3(64 * kFwdWaves), 0, s,
                           op->F.p, op->ftiles.p, op->nftiles, op->fwd_off.p, op->fwd_cols.p, op->leaf_pos.p,
                           op->leaf_n.p, op->perm.p, x, op->poff.p, w.p);
      }
      {
        ScopedTiming tm(op, s, K_REDUCE_FWD);
        hipLaunchKernelGGL(op->kind == 0 ? k_reduce_segments<0> : k_reduce_segments<1>, dim3((unsigned)((op->nxh + 255) / 256)), dim3(256), 0, s, w.p,
                           op->poff.p, op->out_seg.p, op->seg_start.p, op->seg_leaf0.p, op->seg_nleaf.p, op->seg_col.p,
                           op->nxh, w.xh);
      }
    }
    if (op->nfactiles > 0) {
      ScopedTiming tm(op, s, K_FACTOR_IN);
      hipLaunchKernelGGL(k_factor_in, dim3((unsigned)((op->nfactiles + kCoupWaves - 1) / kCoupWaves)),
                         dim3(64 * kCoupWaves), 0, s, op->FY.p, op->factiles.p, op->nfactiles, w.xh,
                         w.xh);
    }
    const cd* zsrc = w.xh;
    if (op->sym) {
      if (op->nyh > 0) {
        if (op->nctiles > 0) {
          ScopedTiming tm(op, s, K_SYM_COUPLING);
          hipLaunchKernelGGL(k_coupling_sym, dim3((unsigned)((op->nctiles + kCoupWaves - 1) / kCoupWaves)),
                             dim3(64 * kCoupWaves), 0, s, op->S.p, op->stiles.p, op->nctiles, op->csrc.p,
                             w.xh, w.part, w.tpart);
        }
        {
          ScopedTiming tm(op, s, K_SYM_REDUCE);
          hipLaunchKernelGGL(k_reduce_sym, dim3((unsigned)((op->nyh + 255) / 256)), dim3(256), 0, s, w.part,
                             w.tpart, op->yh_grp.p, op->grp_start.p, op->grp_t0.p, op->grp_nt.p, op->grp_s0.p,
                             op->grp_ns.p, op->tsrc.p, op->nyh, w.yh);
        }
        zsrc = w.yh;
      }
      {
        ScopedTiming tm(op, s, K_SYM_BACKWARD);
        hipLaunchKernelGGL(k_backward_sym, dim3(nl), dim3(64 * kSymBwdWaves), 0, s, op->B.p, op->bwd_off.p,
                           op->bwd_cols.p, op->bwd_tcol.p, op->td_off.p, op->zoff.p, op->zmap.p, op->leaf_pos.p,
                           op->leaf_n.p, op->perm.p, zsrc, x, y, w.td, nl);
      }
      if (op->tdtot > 0) {
        ScopedTiming tm(op, s, K_SYM_FINISH);
        hipLaunchKernelGGL(k_finish_sym, dim3(nl), dim3(64), 0, s, op->fin_off.p, op->fin_cnt.p, op->fsrc.p,
                           op->leaf_pos.p, op->leaf_n.p, op->perm.p, w.td, y);
      }
      continue;
    }
    if (op->kind == 0 && op->nctiles > 0) {
      {
        ScopedTiming tm(op, s, K_COUPLING);
        hipLaunchKernelGGL(k_coupling, dim3((unsigned)((op->nctiles + kCoupWaves - 1) / kCoupWaves)),
                           dim3(64 * kCoupWaves), 0, s, op->S.p, op->ctiles.p, op->nctiles, op->cblk.p, w.xh,
                           w.part);
      }
      {
        ScopedTiming tm(op, s, K_REDUCE_COUP);
        hipLaunchKernelGGL(k_reduce_coupling, dim3((unsigned)((op->nyh + 255) / 256)), dim3(256), 0, s,
                           w.part, op->yh_grp.p, op->grp_start.p, op->grp_t0.p, op->grp_nt.p, op->nyh,
                           w.yh);
      }
      zsrc = w.yh;
    }
    {
      ScopedTiming tm(op, s, K_BACKWARD);
      hipLaunchKernelGGL(op->kind == 0 ? k_backward<0> : k_backward<1>, dim3(nl), dim3(64 * kBwdWaves), 0, s, op->B.p, op->bwd_off.p, op->bwd_cols.p,
                         op->zoff.p, op->zmap.p, op->leaf_pos.p, op->leaf_n.p, op->perm.p, zsrc, x, y, nl);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(UHM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return UHM_OK;
}

}  // namespace

extern "C" {

int uhm_op_info_get(const uhm_op* op, uhm_op_info* info) {
  if (!op || !info) return fail(UHM_EINVAL, "null argument");
  *info = op->info;
  int64_t off[6];
  info->scratch_bytes = (op->lp || !is_c128(op->storage)) ? 0 : fp64_ws_layout(op, off) * (int64_t)sizeof(cd);
  return UHM_OK;
}

int uhm_set_timing(uhm_op* op, int enabled) {
  if (!op) return fail(UHM_EINVAL, "null operator");
  for (auto& e : op->pending) {
    op->free_events.push_back(e.a);
    op->free_events.push_back(e.b);
  }
  op->pending.clear();
  op->timers.clear();
  for (int k = 0; k < K_COUNT; ++k) op->timers.push_back({kKernelNames[k], 0.0, 0});
  op->timing = enabled != 0;
  return UHM_OK;
}

int uhm_kernel_times(uhm_op* op, const char** names, double* total_ms, int64_t* launches, int32_t cap) {
  if (!op) return fail(UHM_EINVAL, "null operator");
  if (op->timers.empty())
    for (int k = 0; k < K_COUNT; ++k) op->timers.push_back({kKernelNames[k], 0.0, 0});
  for (auto& e : op->pending) {
    UHM_HIP(hipEventSynchronize(e.b));
    float ms = 0.f;
    UHM_HIP(hipEventElapsedTime(&ms, e.a, e.b));
    op->timers[e.kernel].total_ms += ms;
    op->timers[e.kernel].launches += 1;
    op->free_events.push_back(e.a);
    op->free_events.push_back(e.b);
  }
  op->pending.clear();
  const int32_t nk = (int32_t)op->timers.size();
  for (int32_t k = 0; k < std::min(nk, cap); ++k) {
    if (names) names[k] = op->timers[k].name;
    if (total_ms) total_ms[k] = op->timers[k].total_ms;
    if (launches) launches[k] = op->timers[k].launches;
  }
  return nk;
}

void uhm_free(uhm_op* op) { delete op; }

}  // extern "C"
