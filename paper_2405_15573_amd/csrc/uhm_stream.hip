// Streaming single-RHS forms of the uniform H-matrix product in low precision: the layout
// and the four stages of the complex128 product (forward panels, row-chunked couplings,
// leaf-owned backward panels with the near field; Algorithm 6, section 4.4), with the
// operator stored in complex64 (8 bytes per element) or as (re, im) bfloat16 pairs
// (4 bytes), FP32 arithmetic, complex64 vectors.
//
// One lane per panel column (forward) or row (coupling, backward) streams the operator
// once per product; nothing is padded to matrix-core tile widths, so a single right-hand
// side costs the operator's bytes and no more.  Several right-hand sides run one after
// another.  The upload builds the complex128 layout and converts it on the device, so the
// two forms share every index array with the complex128 product.
#include "uhm_internal.h"

namespace uhm_detail {
namespace {

using cf = float2;
typedef float v2f __attribute__((ext_vector_type(2)));

// Workgroups are dealt round-robin over the 8 XCDs: give each XCD a contiguous range of
// leaves, whose shared ancestors' rank-space values then stay in that XCD's L2.
__device__ __forceinline__ int xcd_leaf(int bid, int nb) {
  const int q = nb >> 3, r = nb & 7, x = bid & 7, k = bid >> 3;
  return x * q + min(x, r) + k;
}

// A complex element as two bfloat16 values in one 32-bit word: re in the low half.
struct bfp {
  uint32_t v;
};

__device__ __forceinline__ cf sload(const cf* p) {
  const v2f v = __builtin_nontemporal_load(reinterpret_cast<const v2f*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ cf sload(const bfp* p) {
  const uint32_t u = __builtin_nontemporal_load(&p->v);
  return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

// FP64 -> FP32 (round to nearest) -> bfloat16 (round to nearest, ties to even); the value as
// the upper 16 bits of a float word.
__device__ __forceinline__ uint32_t bf16_bits(double d) {
  const uint32_t u = __float_as_uint((float)d);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__global__ __launch_bounds__(256) void k_s_to_c64(const cd* __restrict__ a, int64_t n, cf* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) out[q] = make_float2((float)a[q].x, (float)a[q].y);
}
__global__ __launch_bounds__(256) void k_s_to_bf16(const cd* __restrict__ a, int64_t n, bfp* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) out[q].v = bf16_bits(a[q].x) | (bf16_bits(a[q].y) << 16);
}

// Forward transform: one wave per 64-column tile of a leaf's panel, lane c accumulating
// conj(F[i,c]) x_i over the leaf's rows (x uniform over the wave: scalar loads).
template <class E>
__global__ __launch_bounds__(64 * kFwdWaves) void k_s_forward(const E* __restrict__ F, const int2* __restrict__ ftiles,
                                                              int32_t ntiles, const int64_t* __restrict__ fwd_off,
                                                              const int32_t* __restrict__ fwd_cols,
                                                              const int32_t* __restrict__ leaf_pos,
                                                              const int32_t* __restrict__ leaf_n,
                                                              const int32_t* __restrict__ perm, const cf* __restrict__ x,
                                                              const int64_t* __restrict__ poff, cf* __restrict__ p) {
  const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * kFwdWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int2 lt = ftiles[tile];
  const int leaf = lt.x, j = lt.y;
  const int n = leaf_n[leaf];
  const int wj = min(kTile, fwd_cols[leaf] - kTile * j);
  if (lane >= wj) return;
  const E* q = F + fwd_off[leaf] + (int64_t)kTile * j * n + lane;
  const int32_t* px = perm + leaf_pos[leaf];
  float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
  int i = 0;
  for (; i + 8 <= n; i += 8) {
    cf v[8], xv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = sload(&q[(i + k) * wj]);
#pragma unroll
    for (int k = 0; k < 8; ++k) xv[k] = x[px[i + k]];
#pragma unroll
    for (int k = 0; k < 8; k += 2) {
      re0 = fmaf(v[k].x, xv[k].x, fmaf(v[k].y, xv[k].y, re0));
      im0 = fmaf(v[k].x, xv[k].y, fmaf(-v[k].y, xv[k].x, im0));
      re1 = fmaf(v[k + 1].x, xv[k + 1].x, fmaf(v[k + 1].y, xv[k + 1].y, re1));
      im1 = fmaf(v[k + 1].x, xv[k + 1].y, fmaf(-v[k + 1].y, xv[k + 1].x, im1));
    }
  }
  for (; i < n; ++i) {
    const cf v = sload(&q[i * wj]), xv = x[px[i]];
    re0 = fmaf(v.x, xv.x, fmaf(v.y, xv.y, re0));
    im0 = fmaf(v.x, xv.y, fmaf(-v.y, xv.x, im0));
  }
  p[poff[leaf] + kTile * j + lane] = make_float2(re0 + re1, im0 + im1);
}

// out[e] = sum over the leaves of e's segment of p[leaf][col + e - start], in leaf order.
__global__ __launch_bounds__(256) void k_s_reduce_segments(const cf* __restrict__ p, const int64_t* __restrict__ poff,
                                                           const int32_t* __restrict__ out_seg,
                                                           const int64_t* __restrict__ seg_start,
                                                           const int32_t* __restrict__ seg_leaf0,
                                                           const int32_t* __restrict__ seg_nleaf,
                                                           const int32_t* __restrict__ seg_col, int64_t nout,
                                                           cf* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  const int s = out_seg[e];
  const int col = seg_col[s] + (int)(e - seg_start[s]);
  const int l0 = seg_leaf0[s], nl = seg_nleaf[s];
  float re = 0.f, im = 0.f;
  int q = 0;
  for (; q + 8 <= nl; q += 8) {
    int64_t o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = poff[l0 + q + k];
    cf v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = p[o[k] + col];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      re += v[k].x;
      im += v[k].y;
    }
  }
  for (; q < nl; ++q) {
    const cf v = p[poff[l0 + q] + col];
    re += v.x;
    im += v.y;
  }
  out[e] = make_float2(re, im);
}

// part[tile][r] = sum_c S_chunk[r, c] xh[src(c)] over the tile's columns, one lane per row
// (xh uniform over the wave: scalar loads).
template <class E>
__global__ __launch_bounds__(64 * kCoupWaves) void k_s_coupling(const E* __restrict__ S, const CoupTile* __restrict__ tiles,
                                                                int32_t ntiles, const int2* __restrict__ cblk,
                                                                const cf* __restrict__ xh, cf* __restrict__ part) {
  const int tile = __builtin_amdgcn_readfirstlane(blockIdx.x * kCoupWaves + (threadIdx.x >> 6));
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const CoupTile T = tiles[tile];
  float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
  const int h = T.h;
  const bool act = lane < h;
  const E* col = S + T.s_base + (act ? lane : 0);
  int b = T.first_blk, j = T.first_col, rem = T.ncols;
  while (rem > 0) {
    const int2 bl = cblk[b];
    const int cnt = min(bl.x - j, rem);
    const cf* xv = xh + bl.y + j;
    int q = 0;
    for (; q + 8 <= cnt; q += 8) {
      cf sv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) sv[k] = sload(&col[(int64_t)(q + k) * h]);
#pragma unroll
      for (int k = 0; k < 8; k += 2) {
        const cf x0 = xv[q + k], x1 = xv[q + k + 1];
        re0 = fmaf(sv[k].x, x0.x, fmaf(-sv[k].y, x0.y, re0));
        im0 = fmaf(sv[k].x, x0.y, fmaf(sv[k].y, x0.x, im0));
        re1 = fmaf(sv[k + 1].x, x1.x, fmaf(-sv[k + 1].y, x1.y, re1));
        im1 = fmaf(sv[k + 1].x, x1.y, fmaf(sv[k + 1].y, x1.x, im1));
      }
    }
    for (; q < cnt; ++q) {
      const cf s0 = sload(&col[(int64_t)q * h]), x0 = xv[q];
      re0 = fmaf(s0.x, x0.x, fmaf(-s0.y, x0.y, re0));
      im0 = fmaf(s0.x, x0.y, fmaf(s0.y, x0.x, im0));
    }
    col += (int64_t)cnt * h;
    rem -= cnt;
    ++b;
    j = 0;
  }
  if (act) part[(int64_t)tile * kRowChunk + lane] = make_float2(re0 + re1, im0 + im1);
}

// yh[e] = sum over the tiles of e's row chunk of part[t][r(e)], tiles in column order.
__global__ __launch_bounds__(256) void k_s_reduce_coupling(const cf* __restrict__ part, const int32_t* __restrict__ yh_grp,
                                                           const int64_t* __restrict__ grp_start,
                                                           const int32_t* __restrict__ grp_t0,
                                                           const int32_t* __restrict__ grp_nt, int64_t nout,
                                                           cf* __restrict__ yh) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nout) return;
  const int g = yh_grp[e];
  const int r = (int)(e - grp_start[g]);
  const int t0 = grp_t0[g], nt = grp_nt[g];
  float re = 0.f, im = 0.f;
  for (int t = 0; t < nt; ++t) {
    const cf v = part[(int64_t)(t0 + t) * kRowChunk + r];
    re += v.x;
    im += v.y;
  }
  yh[e] = make_float2(re, im);
}

// y|_lambda = B_lambda z_lambda, z gathered into LDS from the rank-space vector (index >= 0)
// or from the user-order input (index = -1 - user index); one lane per leaf row, the columns
// split over the waves, partial sums added in wave order.
template <class E>
__global__ __launch_bounds__(64 * kBwdWaves) void k_s_backward(const E* __restrict__ B, const int64_t* __restrict__ bwd_off,
                                                               const int32_t* __restrict__ bwd_cols,
                                                               const int64_t* __restrict__ zoff,
                                                               const int32_t* __restrict__ zmap,
                                                               const int32_t* __restrict__ leaf_pos,
                                                               const int32_t* __restrict__ leaf_n,
                                                               const int32_t* __restrict__ perm, const cf* __restrict__ yh,
                                                               const cf* __restrict__ x, cf* __restrict__ y,
                                                               int nleaves) {
  const int leaf = xcd_leaf(blockIdx.x, nleaves);
  const int K = bwd_cols[leaf], n = leaf_n[leaf];
  __shared__ cf zs[kBwdChunk];
  __shared__ cf red[kBwdWaves][kLeafMax];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const E* Bl = B + bwd_off[leaf];
  const int32_t* zm = zmap + zoff[leaf];
  float re0 = 0.f, im0 = 0.f, re1 = 0.f, im1 = 0.f;
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
      const E* col = Bl + (int64_t)(c0 + a) * n + lane;
      int c = a;
      for (; c + 8 <= e; c += 8, col += 8 * n) {
        cf bv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) bv[k] = sload(&col[k * n]);
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
          const cf z0 = zs[c + k], z1 = zs[c + k + 1];
          re0 = fmaf(bv[k].x, z0.x, fmaf(-bv[k].y, z0.y, re0));
          im0 = fmaf(bv[k].x, z0.y, fmaf(bv[k].y, z0.x, im0));
          re1 = fmaf(bv[k + 1].x, z1.x, fmaf(-bv[k + 1].y, z1.y, re1));
          im1 = fmaf(bv[k + 1].x, z1.y, fmaf(bv[k + 1].y, z1.x, im1));
        }
      }
      for (; c < e; ++c, col += n) {
        const cf b0 = sload(col), z0 = zs[c];
        re0 = fmaf(b0.x, z0.x, fmaf(-b0.y, z0.y, re0));
        im0 = fmaf(b0.x, z0.y, fmaf(b0.y, z0.x, im0));
      }
    }
  }
  red[w][lane] = make_float2(re0 + re1, im0 + im1);
  __syncthreads();
  if (w == 0 && act) {
    float sr = 0.f, si = 0.f;
    for (int q = 0; q < kBwdWaves; ++q) {
      sr += red[q][lane].x;
      si += red[q][lane].y;
    }
    y[perm[leaf_pos[leaf] + lane]] = make_float2(sr, si);
  }
}

// Convert a complex128 device array to the form's element type, then drop it.
int compact(DevArray<cd>& a, DevArray<unsigned char>& out, int storage, hipStream_t s) {
  const int64_t n = a.n;
  const int64_t eb = storage == UHM_C64_STREAM ? 8 : 4;
  int rc;
  if ((rc = out.alloc(std::max<int64_t>(1, n) * eb))) return rc;
  if (n > 0) {
    const dim3 g((unsigned)((n + 255) / 256));
    if (storage == UHM_C64_STREAM)
      hipLaunchKernelGGL(k_s_to_c64, g, dim3(256), 0, s, a.p, n, reinterpret_cast<cf*>(out.p));
    else
      hipLaunchKernelGGL(k_s_to_bf16, g, dim3(256), 0, s, a.p, n, reinterpret_cast<bfp*>(out.p));
  }
  UHM_HIP(hipGetLastError());
  UHM_HIP(hipStreamSynchronize(s));
  return a.alloc(0);
}

template <class E>
int launch_stream(uhm_op* op, const cf* x, cf* y, hipStream_t s) {
  const E* F = reinterpret_cast<const E*>(op->Fs.p);
  const E* S = reinterpret_cast<const E*>(op->Ss.p);
  const E* B = reinterpret_cast<const E*>(op->Bs.p);
  cf* p = reinterpret_cast<cf*>(op->ws_p.p);
  cf* xh = reinterpret_cast<cf*>(op->ws_xh.p);
  cf* part = reinterpret_cast<cf*>(op->ws_part.p);
  cf* yh = reinterpret_cast<cf*>(op->ws_yh.p);
  if (op->nxh > 0) {
    {
      ScopedTiming tm(op, s, K_FORWARD);
      hipLaunchKernelGGL(k_s_forward<E>, dim3((unsigned)((op->nftiles + kFwdWaves - 1) / kFwdWaves)),
                         dim3(64 * kFwdWaves), 0, s, F, op->ftiles.p, op->nftiles, op->fwd_off.p, op->fwd_cols.p,
                         op->leaf_pos.p, op->leaf_n.p, op->perm.p, x, op->poff.p, p);
    }
    {
      ScopedTiming tm(op, s, K_REDUCE_FWD);
      hipLaunchKernelGGL(k_s_reduce_segments, dim3((unsigned)((op->nxh + 255) / 256)), dim3(256), 0, s, p, op->poff.p,
                         op->out_seg.p, op->seg_start.p, op->seg_leaf0.p, op->seg_nleaf.p, op->seg_col.p, op->nxh, xh);
    }
  }
  if (op->nctiles > 0) {
    {
      ScopedTiming tm(op, s, K_COUPLING);
      hipLaunchKernelGGL(k_s_coupling<E>, dim3((unsigned)((op->nctiles + kCoupWaves - 1) / kCoupWaves)),
                         dim3(64 * kCoupWaves), 0, s, S, op->ctiles.p, op->nctiles, op->cblk.p, xh, part);
    }
    {
      ScopedTiming tm(op, s, K_REDUCE_COUP);
      hipLaunchKernelGGL(k_s_reduce_coupling, dim3((unsigned)((op->nyh + 255) / 256)), dim3(256), 0, s, part,
                         op->yh_grp.p, op->grp_start.p, op->grp_t0.p, op->grp_nt.p, op->nyh, yh);
    }
  }
  {
    ScopedTiming tm(op, s, K_BACKWARD);
    hipLaunchKernelGGL(k_s_backward<E>, dim3((unsigned)op->nleaves), dim3(64 * kBwdWaves), 0, s, B, op->bwd_off.p,
                       op->bwd_cols.p, op->zoff.p, op->zmap.p, op->leaf_pos.p, op->leaf_n.p, op->perm.p, yh, x, y,
                       op->nleaves);
  }
  return UHM_OK;
}

}  // namespace

int stream_compact(uhm_op* op, hipStream_t s) {
  int rc;
  if ((rc = compact(op->F, op->Fs, op->storage, s)) || (rc = compact(op->S, op->Ss, op->storage, s)) ||
      (rc = compact(op->B, op->Bs, op->storage, s)))
    return rc;
  return UHM_OK;
}

int stream_matvec(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, hipStream_t s) {
  int rc = grow_workspace_fp64(op);
  if (rc) return rc;
  for (int32_t r = 0; r < nrhs; ++r) {
    const cf* x = static_cast<const cf*>(X) + (int64_t)r * ldx;
    cf* y = static_cast<cf*>(Y) + (int64_t)r * ldy;
    rc = op->storage == UHM_C64_STREAM ? launch_stream<cf>(op, x, y, s) : launch_stream<bfp>(op, x, y, s);
    if (rc) return rc;
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(UHM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return UHM_OK;
}

}  // namespace uhm_detail
