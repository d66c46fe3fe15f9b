// Low-precision storage forms of the uniform H-matrix product: complex64 (FP32 MFMA) and
// (re, im) bfloat16 pairs (BF16 MFMA), FP32 accumulation, 1 to 64 right-hand sides per
// pass.  The three stages of Algorithm 6 (section 4.4) become batched complex GEMMs:
//
//   forward   P_lambda = F_lambda^* X_lambda   (C_lambda x r; K = leaf rows)
//   coupling  Y^_tau   = [S_b ...] X^cat       (l_tau x r;    K = sum_sigma l_sigma)
//   backward  Y_lambda = B_lambda Z_lambda     (n_lambda x r; K = ancestor ranks + near field)
//
// with the same per-leaf panels, row-chunked couplings and deterministic reductions as the
// FP64 path.  The operator panels (the "A" operands) are streamed from HBM once per product
// in a fragment-major layout: for every 16-row m-tile and every k-block, each lane's
// KPL consecutive k-values of its row are one contiguous 32-byte chunk (real parts, then
// imaginary parts), so a wavefront loads a contiguous run with 16-byte lane loads.  The
// vector operand (the "B" operand: gathered rows of x, u_sigma or u_tau) is staged in LDS
// in FP32 (complex64 path) or as bf16 hi + lo parts (bf16 path), so that in the bf16 form
// the only bf16 rounding is that of the stored operator.
//
// MFMA lane layouts (checked on gfx950):
//   v_mfma_f32_16x16x4_f32:  A lane l = A[l%16][l/16], B lane l = B[l/16][l%16]
//   v_mfma_f32_16x16x32_bf16: A lane l = A[l%16][8(l/16)+t], B lane l = B[8(l/16)+t][l%16]
//   both: accumulator register v of lane l = C[4(l/16)+v][l%16].
// The k index inside one instruction may be any permutation shared by A and B; here lane
// group g = l/16 owns the k-values g*KPL .. g*KPL+KPL-1 of the k-block.
#include "uhm_internal.h"

#include <climits>
#include <complex>

namespace uhm_detail {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
using cf = float2;

constexpr int kLpWaves = 4;
constexpr int kLpZ = 64;          // k-rows of the B operand staged in LDS per round
constexpr int kLpCoupK = 1024;    // coupling tile width in columns (multiple of kLpZ)
constexpr int kLpRmax = 64;       // right-hand sides per pass
constexpr int32_t kZero = INT_MIN;  // gather-map entry for a zero (padding) column

template <int ST>
struct Frag;
template <>
struct Frag<UHM_C64> {
  static constexpr int KB = 16, KPL = 4;
};
template <>
struct Frag<UHM_BF16PAIR> {
  static constexpr int KB = 32, KPL = 8;
};

// LDS image of the B operand for one round of kLpZ k-rows and R <= 64 columns.
constexpr int kRS = kLpRmax + 4;   // complex64 row stride (keeps lane groups on other banks)
constexpr int kZT = kLpZ + 8;      // bf16 plane row stride (per column j)
struct LdsF32 {
  cf z[kLpZ * kRS];
};
struct LdsBf16 {
  __bf16 re_hi[kLpRmax * kZT], re_lo[kLpRmax * kZT], im_hi[kLpRmax * kZT], im_lo[kLpRmax * kZT];
};

__device__ __forceinline__ void lds_put(LdsF32& L, int k, int j, cf v) { L.z[k * kRS + j] = v; }
__device__ __forceinline__ void lds_put(LdsBf16& L, int k, int j, cf v) {
  const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
  L.re_hi[j * kZT + k] = rh;
  L.re_lo[j * kZT + k] = (__bf16)(v.x - (float)rh);
  L.im_hi[j * kZT + k] = ih;
  L.im_lo[j * kZT + k] = (__bf16)(v.y - (float)ih);
}

// One lane's A chunk of a k-block: KPL complex values of its row.
struct ChunkF32 {
  v4f re, im;
};
struct ChunkBf16 {
  v8bf re, im;
};

__device__ __forceinline__ void load_chunk(const uint4* p, bool act, ChunkF32& c) {
  if (act) {
    const uint4 a = p[0], b = p[1];
    c.re = v4f{__uint_as_float(a.x), __uint_as_float(a.y), __uint_as_float(a.z), __uint_as_float(a.w)};
    c.im = v4f{__uint_as_float(b.x), __uint_as_float(b.y), __uint_as_float(b.z), __uint_as_float(b.w)};
  } else {
    c.re = v4f{0.f, 0.f, 0.f, 0.f};
    c.im = c.re;
  }
}
__device__ __forceinline__ void load_chunk(const uint4* p, bool act, ChunkBf16& c) {
  uint4 a = make_uint4(0, 0, 0, 0), b = a;
  if (act) {
    a = p[0];
    b = p[1];
  }
  c.re = __builtin_bit_cast(v8bf, a);
  c.im = __builtin_bit_cast(v8bf, b);
}

// acc_r/acc_i[nt] += A_chunk (16 rows x one k-block) * B (k-block rows of the LDS round).
template <int NT>
__device__ __forceinline__ void mma_block(const ChunkF32& a, const LdsF32& L, int kk0, int g, int i, v4f* cr, v4f* ci) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = kk0 + g * 4 + t;
    const float ar = a.re[t], ai = a.im[t], nai = -a.im[t];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const cf b = L.z[k * kRS + nt * 16 + i];
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b.x, cr[nt], 0, 0, 0);
      cr[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai, b.y, cr[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b.y, ci[nt], 0, 0, 0);
      ci[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b.x, ci[nt], 0, 0, 0);
    }
  }
}

template <int NT>
__device__ __forceinline__ void mma_block(const ChunkBf16& a, const LdsBf16& L, int kk0, int g, int i, v4f* cr,
                                          v4f* ci) {
  uint4 neg = __builtin_bit_cast(uint4, a.im);
  neg.x ^= 0x80008000u;
  neg.y ^= 0x80008000u;
  neg.z ^= 0x80008000u;
  neg.w ^= 0x80008000u;
  const v8bf nai = __builtin_bit_cast(v8bf, neg);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int o = (nt * 16 + i) * kZT + kk0 + g * 8;
    const v8bf brh = *reinterpret_cast<const v8bf*>(&L.re_hi[o]);
    const v8bf brl = *reinterpret_cast<const v8bf*>(&L.re_lo[o]);
    const v8bf bih = *reinterpret_cast<const v8bf*>(&L.im_hi[o]);
    const v8bf bil = *reinterpret_cast<const v8bf*>(&L.im_lo[o]);
    cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, brh, cr[nt], 0, 0, 0);
    cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, brl, cr[nt], 0, 0, 0);
    cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai, bih, cr[nt], 0, 0, 0);
    cr[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai, bil, cr[nt], 0, 0, 0);
    ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, bih, ci[nt], 0, 0, 0);
    ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, bil, ci[nt], 0, 0, 0);
    ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.im, brh, ci[nt], 0, 0, 0);
    ci[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.im, brl, ci[nt], 0, 0, 0);
  }
}

template <int ST>
using LdsOf = typename std::conditional<ST == UHM_C64, LdsF32, LdsBf16>::type;
template <int ST>
using ChunkOf = typename std::conditional<ST == UHM_C64, ChunkF32, ChunkBf16>::type;

// Store the 16 x (16 NT) accumulator tile: row r = 4g + v (< hm), column j = 16 nt + i (< R).
template <int NT>
__device__ __forceinline__ void store_tile(cf* out, int64_t row0, int hm, int R, int g, int i, const v4f* cr,
                                           const v4f* ci) {
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * g + v;
      if (r < hm) out[(row0 + r) * R + nt * 16 + i] = make_float2(cr[nt][v], ci[nt][v]);
    }
}

// ---------------------------------------------------------------- kernels

// Xc[pos][j] = x[perm[pos] + j ldx] (cluster order, row-major, R columns, zero beyond r).
__global__ __launch_bounds__(256) void k_lp_gather(const cf* __restrict__ x, int64_t ldx, int r, int R,
                                                   const int32_t* __restrict__ perm, int64_t n, cf* __restrict__ Xc) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n * R) return;
  const int64_t pos = q / R;
  const int j = (int)(q - pos * R);
  Xc[q] = j < r ? x[perm[pos] + (int64_t)j * ldx] : make_float2(0.f, 0.f);
}

__global__ __launch_bounds__(256) void k_lp_scatter(const cf* __restrict__ Yc, int r, int R, const int32_t* __restrict__ perm,
                                                    int64_t n, cf* __restrict__ y, int64_t ldy) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= n * (int64_t)r) return;
  const int j = (int)(q / n);
  const int64_t pos = q - (int64_t)j * n;
  y[perm[pos] + (int64_t)j * ldy] = Yc[pos * R + j];
}

// P_lambda = F_lambda^* X_lambda for every leaf (one workgroup per leaf).
template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lp_forward(
    const uint4* __restrict__ F, const int64_t* __restrict__ f_off, const int32_t* __restrict__ f_M,
    const int32_t* __restrict__ f_nkb, const int32_t* __restrict__ leaf_pos, const int32_t* __restrict__ leaf_n,
    const int64_t* __restrict__ poff, const cf* __restrict__ Xc, int R, cf* __restrict__ p) {
  using F_ = Frag<ST>;
  __shared__ LdsOf<ST> L;
  const int leaf = blockIdx.x;
  const int M = f_M[leaf];
  if (M == 0) return;
  const int n = leaf_n[leaf], nkb = f_nkb[leaf];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, i = lane & 15;
  const int K = nkb * F_::KB;  // <= 64
  for (int q = t; q < K * R; q += 64 * kLpWaves) {
    const int k = q / R, j = q - k * R;
    lds_put(L, k, j, k < n ? Xc[(int64_t)(leaf_pos[leaf] + k) * R + j] : make_float2(0.f, 0.f));
  }
  __syncthreads();
  const uint4* base = F + f_off[leaf];
  const int nmt = (M + 15) >> 4;
  for (int mt = w; mt < nmt; mt += kLpWaves) {
    const int hm = min(16, M - 16 * mt);
    const uint4* tile = base + (int64_t)mt * nkb * 8 * 16;
    v4f cr[NT], ci[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) cr[nt] = ci[nt] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < nkb; ++kb) {
      ChunkOf<ST> a;
      load_chunk(tile + (int64_t)kb * 8 * hm + 2 * (g * hm + i), i < hm, a);
      mma_block<NT>(a, L, kb * F_::KB, g, i, cr, ci);
    }
    store_tile<NT>(p, poff[leaf] + 16 * mt, hm, R, g, i, cr, ci);
  }
}

// xh[e][j] = sum over the leaves of the segment of p[poff[leaf] + col + e - start][j].
__global__ __launch_bounds__(256) void k_lp_reduce_segments(const cf* __restrict__ p, int R, const int64_t* __restrict__ poff,
                                                            const int32_t* __restrict__ out_seg,
                                                            const int64_t* __restrict__ seg_start,
                                                            const int32_t* __restrict__ seg_leaf0,
                                                            const int32_t* __restrict__ seg_nleaf,
                                                            const int32_t* __restrict__ seg_col, int64_t nout,
                                                            cf* __restrict__ xh) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nout * R) return;
  const int64_t e = q / R;
  const int j = (int)(q - e * R);
  const int s = out_seg[e];
  const int col = seg_col[s] + (int)(e - seg_start[s]);
  const int l0 = seg_leaf0[s], nl = seg_nleaf[s];
  float re = 0.f, im = 0.f;
  for (int qq = 0; qq < nl; ++qq) {
    const cf v = p[(poff[l0 + qq] + col) * R + j];
    re += v.x;
    im += v.y;
  }
  xh[q] = make_float2(re, im);
}

struct LpCoupTile {
  int64_t base;     // uint4 offset of the chunk panel (all its m-tiles)
  int64_t csrc;     // offset of the chunk's first column in the column-source map
  int32_t h;        // rows of the chunk (<= 64)
  int32_t nkb_all;  // k-blocks of the chunk panel (stride between its m-tiles)
  int32_t kb0;      // first k-block of this tile
  int32_t nkb;      // k-blocks in this tile
};

// Partial u_tau of one coupling tile (workgroup; wave w = m-tile w of the chunk).
template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lp_coupling(const uint4* __restrict__ S,
                                                               const LpCoupTile* __restrict__ tiles,
                                                               const int32_t* __restrict__ colsrc,
                                                               const cf* __restrict__ xh, int R,
                                                               cf* __restrict__ part) {
  using F_ = Frag<ST>;
  __shared__ LdsOf<ST> L;
  const LpCoupTile T = tiles[blockIdx.x];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, i = lane & 15;
  const int nmt = (T.h + 15) >> 4;
  const int hm = min(16, T.h - 16 * w);
  const uint4* tile = S + T.base + (int64_t)w * T.nkb_all * 8 * 16;
  v4f cr[NT], ci[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) cr[nt] = ci[nt] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int KBR = kLpZ / F_::KB;  // k-blocks per LDS round
  for (int kb = 0; kb < T.nkb; kb += KBR) {
    const int nk = min(KBR, T.nkb - kb) * F_::KB;
    const int64_t c0 = T.csrc + (int64_t)(T.kb0 + kb) * F_::KB;
    __syncthreads();
    for (int q = t; q < nk * R; q += 64 * kLpWaves) {
      const int k = q / R, j = q - k * R;
      const int32_t src = colsrc[c0 + k];
      lds_put(L, k, j, src >= 0 ? xh[(int64_t)src * R + j] : make_float2(0.f, 0.f));
    }
    __syncthreads();
    if (w < nmt) {
      for (int b = 0; b < nk / F_::KB; ++b) {
        ChunkOf<ST> a;
        load_chunk(tile + (int64_t)(T.kb0 + kb + b) * 8 * hm + 2 * (g * hm + i), i < hm, a);
        mma_block<NT>(a, L, b * F_::KB, g, i, cr, ci);
      }
    }
  }
  if (w < nmt) store_tile<NT>(part, (int64_t)blockIdx.x * 64 + 16 * w, hm, R, g, i, cr, ci);
}

__global__ __launch_bounds__(256) void k_lp_reduce_coupling(const cf* __restrict__ part, int R,
                                                            const int32_t* __restrict__ yh_grp,
                                                            const int64_t* __restrict__ grp_start,
                                                            const int32_t* __restrict__ grp_t0,
                                                            const int32_t* __restrict__ grp_nt, int64_t nout,
                                                            cf* __restrict__ yh) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nout * R) return;
  const int64_t e = q / R;
  const int j = (int)(q - e * R);
  const int gi = yh_grp[e];
  const int r = (int)(e - grp_start[gi]);
  const int t0 = grp_t0[gi], nt = grp_nt[gi];
  float re = 0.f, im = 0.f;
  for (int tt = 0; tt < nt; ++tt) {
    const cf v = part[((int64_t)(t0 + tt) * 64 + r) * R + j];
    re += v.x;
    im += v.y;
  }
  yh[q] = make_float2(re, im);
}

// Y_lambda = B_lambda Z_lambda per leaf; Z gathered from yh (index >= 0), from the
// cluster-ordered input (index = -1 - position) or zero (kZero).
template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lp_backward(
    const uint4* __restrict__ B, const int64_t* __restrict__ b_off, const int32_t* __restrict__ b_nkb,
    const int64_t* __restrict__ zoff, const int32_t* __restrict__ zmap, const int32_t* __restrict__ leaf_pos,
    const int32_t* __restrict__ leaf_n, const cf* __restrict__ yh, const cf* __restrict__ Xc, int R,
    cf* __restrict__ Yc) {
  using F_ = Frag<ST>;
  __shared__ LdsOf<ST> L;
  const int leaf = blockIdx.x;
  const int n = leaf_n[leaf], nkb = b_nkb[leaf];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, i = lane & 15;
  const int nmt = (n + 15) >> 4;
  const int hm = min(16, n - 16 * w);
  const uint4* tile = B + b_off[leaf] + (int64_t)w * nkb * 8 * 16;
  const int32_t* zm = zmap + zoff[leaf];
  v4f cr[NT], ci[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) cr[nt] = ci[nt] = v4f{0.f, 0.f, 0.f, 0.f};
  constexpr int KBR = kLpZ / F_::KB;
  for (int kb = 0; kb < nkb; kb += KBR) {
    const int nk = min(KBR, nkb - kb) * F_::KB;
    __syncthreads();
    for (int q = t; q < nk * R; q += 64 * kLpWaves) {
      const int k = q / R, j = q - k * R;
      const int32_t m = zm[kb * F_::KB + k];
      cf v = make_float2(0.f, 0.f);
      if (m >= 0)
        v = yh[(int64_t)m * R + j];
      else if (m != kZero)
        v = Xc[(int64_t)(-1 - m) * R + j];
      lds_put(L, k, j, v);
    }
    __syncthreads();
    if (w < nmt) {
      for (int b = 0; b < nk / F_::KB; ++b) {
        ChunkOf<ST> a;
        load_chunk(tile + (int64_t)(kb + b) * 8 * hm + 2 * (g * hm + i), i < hm, a);
        mma_block<NT>(a, L, b * F_::KB, g, i, cr, ci);
      }
    }
  }
  if (w < nmt) store_tile<NT>(Yc, (int64_t)leaf_pos[leaf] + 16 * w, hm, R, g, i, cr, ci);
}

}  // namespace

// ---------------------------------------------------------------- host side

struct LowpOp {
  int storage = UHM_C64;
  int KB = 16;
  DevArray<uint4> F, S, B;
  DevArray<int64_t> f_off, poff, b_off, zoff, seg_start, grp_start;
  DevArray<int32_t> f_M, f_nkb, b_nkb, zmap, colsrc, out_seg, seg_leaf0, seg_nleaf, seg_col, yh_grp, grp_t0, grp_nt;
  DevArray<LpCoupTile> ctiles;
  int64_t p_rows = 0, nxh = 0, nyh = 0;
  int32_t nctiles = 0;
  // workspace, sized for R columns
  int wsR = 0;
  DevArray<cf> Xc, Yc, p, xh, part, yh;
};

void lowp_delete(LowpOp* lp) { delete lp; }

namespace {

uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}

// Pack an M x Kp panel (Kp a multiple of KB) given by get(m, k) into fragment-major chunks.
template <int ST, class Get>
int pack_panel(StagerT<uint4>& st, int32_t M, int32_t nkb, Get get) {
  constexpr int KB = Frag<ST>::KB, KPL = Frag<ST>::KPL;
  std::complex<double> v[KPL];
  for (int32_t mt = 0; 16 * mt < M; ++mt) {
    const int32_t hm = std::min(16, M - 16 * mt);
    for (int32_t kb = 0; kb < nkb; ++kb) {
      uint4* dst = st.span((int64_t)8 * hm);
      for (int g = 0; g < 4; ++g)
        for (int32_t i = 0; i < hm; ++i) {
          for (int t = 0; t < KPL; ++t) v[t] = get(16 * mt + i, kb * KB + g * KPL + t);
          uint4* c = dst + 2 * (g * hm + i);
          if (ST == UHM_C64) {
            float re[4], im[4];
            for (int t = 0; t < 4; ++t) {
              re[t] = (float)v[t].real();
              im[t] = (float)v[t].imag();
            }
            std::memcpy(&c[0], re, 16);
            std::memcpy(&c[1], im, 16);
          } else {
            uint16_t re[8], im[8];
            for (int t = 0; t < 8; ++t) {
              re[t] = to_bf16((float)v[t].real());
              im[t] = to_bf16((float)v[t].imag());
            }
            std::memcpy(&c[0], re, 16);
            std::memcpy(&c[1], im, 16);
          }
        }
    }
  }
  return st.err;
}

int64_t panel_chunks(int32_t M, int32_t nkb) { return (int64_t)8 * M * nkb; }  // uint4 units

using C = std::complex<double>;

inline C cget(const double* a, int64_t idx) { return C(a[2 * idx], a[2 * idx + 1]); }

struct SegLp {
  int64_t start;
  int32_t len, leaf0, nleaf, col;
};

template <int ST>
int lowp_upload_t(const uhm_host_operator* h, hipStream_t s, const TreeInfo& T, uhm_op* op, LowpOp* lp) {
  constexpr int KB = Frag<ST>::KB;
  const int32_t nc = h->nclusters;
  const int32_t nl = (int32_t)T.leaves.size();
  int rc;
  std::vector<int64_t> xh_off(nc, -1), yh_off(nc, -1);
  int64_t nxh = 0, nyh = 0;
  for (int32_t c = 0; c < nc; ++c) {
    if (h->rank_col[c] > 0) { xh_off[c] = nxh; nxh += h->rank_col[c]; }
    if (h->rank_row[c] > 0) { yh_off[c] = nyh; nyh += h->rank_row[c]; }
  }
  if (nxh > INT32_MAX / kLpRmax || nyh > INT32_MAX / kLpRmax) return fail(UHM_ENOTSUP, "rank space too large");

  // ---- forward panels: A = F_lambda^* (C_lambda x roundup(n_lambda, KB))
  std::vector<int64_t> f_off(nl), poff(nl);
  std::vector<int32_t> f_M(nl), f_nkb(nl), seg_col_of(nc, -1);
  int64_t ftot = 0, prow = 0;
  for (int32_t i = 0; i < nl; ++i) {
    int32_t Cn = 0;
    for (int32_t a : T.anc[i])
      if (h->rank_col[a] > 0) {
        if (seg_col_of[a] < 0) seg_col_of[a] = Cn;
        Cn += h->rank_col[a];
      }
    f_M[i] = Cn;
    f_nkb[i] = (int32_t)((h->size[T.leaves[i]] + KB - 1) / KB);
    f_off[i] = ftot;
    poff[i] = prow;
    ftot += panel_chunks(Cn, f_nkb[i]);
    prow += Cn;
  }
  if ((rc = lp->F.alloc(ftot))) return rc;
  if (ftot > 0) {
    StagerT<uint4> st;
    if ((rc = st.init(lp->F.p, ftot, s))) return rc;
    std::vector<const double*> colp;  // per panel column: start of the leaf's rows in that basis column
    for (int32_t i = 0; i < nl && !st.err; ++i) {
      const int32_t lf = T.leaves[i];
      const int64_t n = h->size[lf];
      colp.clear();
      for (int32_t a : T.anc[i])
        if (h->rank_col[a] > 0)
          for (int32_t j = 0; j < h->rank_col[a]; ++j)
            colp.push_back(h->V + 2 * (h->V_off[a] + (int64_t)j * h->size[a] + (h->off[lf] - h->off[a])));
      if ((rc = pack_panel<ST>(st, f_M[i], f_nkb[i], [&](int32_t m, int32_t k) -> C {
             return k < n ? std::conj(cget(colp[m], k)) : C(0.0, 0.0);
           })))
        return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = lp->f_off.upload(f_off, s)) || (rc = lp->f_M.upload(f_M, s)) || (rc = lp->f_nkb.upload(f_nkb, s)) ||
      (rc = lp->poff.upload(poff, s)))
    return rc;
  lp->p_rows = prow;
  // segments of u_sigma: sums over the leaves of sigma
  std::vector<SegLp> segs;
  for (int32_t c = 0; c < nc; ++c)
    if (h->rank_col[c] > 0) segs.push_back({xh_off[c], h->rank_col[c], T.leaf_first[c], T.leaf_cnt[c], seg_col_of[c]});
  {
    std::vector<int32_t> out_seg(nxh), l0(segs.size()), nlv(segs.size()), col(segs.size());
    std::vector<int64_t> start(segs.size());
    for (size_t k = 0; k < segs.size(); ++k) {
      const SegLp& sg = segs[k];
      if (sg.leaf0 < 0 || sg.nleaf < 1 || sg.leaf0 + sg.nleaf > nl) return fail(UHM_EINVAL, "layout: segment");
      for (int32_t q = 0; q < sg.nleaf; ++q)
        if (sg.col < 0 || sg.col + sg.len > f_M[sg.leaf0 + q]) return fail(UHM_EINVAL, "layout: segment column");
      for (int32_t j = 0; j < sg.len; ++j) out_seg[sg.start + j] = (int32_t)k;
      start[k] = sg.start;
      l0[k] = sg.leaf0;
      nlv[k] = sg.nleaf;
      col[k] = sg.col;
    }
    if ((rc = lp->out_seg.upload(out_seg, s)) || (rc = lp->seg_start.upload(start, s)) ||
        (rc = lp->seg_leaf0.upload(l0, s)) || (rc = lp->seg_nleaf.upload(nlv, s)) || (rc = lp->seg_col.upload(col, s)))
      return rc;
  }
  lp->nxh = nxh;

  // ---- couplings: row chunks of 64 rows, K padded to KB, tiles of kLpCoupK columns
  std::vector<std::vector<int64_t>> rowblk(nc);
  for (int64_t b = 0; b < h->nadm; ++b) rowblk[h->adm_row[b]].push_back(b);
  std::vector<LpCoupTile> tiles;
  std::vector<int32_t> colsrc, grp_t0, grp_nt, yh_grp(nyh);
  std::vector<int64_t> grp_start;
  int64_t stot = 0;
  struct ChunkJob {
    int32_t tau, r0, h;
    int64_t base, csrc;
    int32_t nkb;
  };
  std::vector<ChunkJob> jobs;
  for (int32_t t = 0; t < nc; ++t) {
    if (rowblk[t].empty()) continue;
    std::sort(rowblk[t].begin(), rowblk[t].end());
    const int32_t lt = h->rank_row[t];
    int64_t K = 0;
    for (int64_t b : rowblk[t]) K += h->rank_col[h->adm_col[b]];
    const int32_t nkb = (int32_t)((K + KB - 1) / KB);
    const int64_t csrc = (int64_t)colsrc.size();
    for (int64_t b : rowblk[t])
      for (int32_t j = 0; j < h->rank_col[h->adm_col[b]]; ++j) colsrc.push_back((int32_t)(xh_off[h->adm_col[b]] + j));
    while ((int64_t)colsrc.size() < csrc + (int64_t)nkb * KB) colsrc.push_back(-1);
    for (int32_t r0 = 0; r0 < lt; r0 += 64) {
      const int32_t hh = std::min(64, lt - r0);
      const int32_t gi = (int32_t)grp_start.size();
      grp_start.push_back(yh_off[t] + r0);
      grp_t0.push_back((int32_t)tiles.size());
      for (int32_t r = 0; r < hh; ++r) yh_grp[yh_off[t] + r0 + r] = gi;
      constexpr int KBT = kLpCoupK / KB;
      for (int32_t kb0 = 0; kb0 < nkb; kb0 += KBT)
        tiles.push_back({stot, csrc, hh, nkb, kb0, std::min(KBT, nkb - kb0)});
      grp_nt.push_back((int32_t)tiles.size() - grp_t0.back());
      jobs.push_back({t, r0, hh, stot, csrc, nkb});
      stot += panel_chunks(hh, nkb);
    }
  }
  if ((rc = lp->S.alloc(stot))) return rc;
  if (stot > 0) {
    StagerT<uint4> st;
    if ((rc = st.init(lp->S.p, stot, s))) return rc;
    std::vector<std::pair<const double*, int64_t>> colp;  // per column: (S_b column start, l_tau)
    for (const ChunkJob& J : jobs) {
      if (st.err) break;
      const int32_t lt = h->rank_row[J.tau];
      colp.clear();
      for (int64_t b : rowblk[J.tau])
        for (int32_t j = 0; j < h->rank_col[h->adm_col[b]]; ++j)
          colp.push_back({h->S + 2 * (h->S_off[b] + (int64_t)j * lt + J.r0), lt});
      const int64_t K = (int64_t)colp.size();
      if ((rc = pack_panel<ST>(st, J.h, J.nkb, [&](int32_t m, int32_t k) -> C {
             return k < K ? cget(colp[k].first, m) : C(0.0, 0.0);
           })))
        return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  for (const LpCoupTile& Tt : tiles) {
    if (Tt.h < 1 || Tt.h > 64 || Tt.base < 0 || Tt.base + panel_chunks(Tt.h, Tt.nkb_all) > stot ||
        Tt.kb0 < 0 || Tt.nkb < 1 || Tt.kb0 + Tt.nkb > Tt.nkb_all || Tt.csrc + (int64_t)Tt.nkb_all * KB > (int64_t)colsrc.size())
      return fail(UHM_EINVAL, "layout: coupling tile");
  }
  for (int32_t v : colsrc)
    if (v >= nxh) return fail(UHM_EINVAL, "layout: coupling column source");
  if ((rc = lp->ctiles.upload(tiles, s)) || (rc = lp->colsrc.upload(colsrc, s)) || (rc = lp->yh_grp.upload(yh_grp, s)) ||
      (rc = lp->grp_start.upload(grp_start, s)) || (rc = lp->grp_t0.upload(grp_t0, s)) ||
      (rc = lp->grp_nt.upload(grp_nt, s)))
    return rc;
  lp->nctiles = (int32_t)tiles.size();
  lp->nyh = nyh;

  // ---- backward panels: ancestor bases then dense blocks; K padded to KB
  std::vector<std::vector<int64_t>> denrow(nc);
  for (int64_t b = 0; b < h->nden; ++b) denrow[h->den_row[b]].push_back(b);
  std::vector<int64_t> b_off(nl), zoff(nl);
  std::vector<int32_t> b_nkb(nl), zmap;
  int64_t btot = 0;
  for (int32_t i = 0; i < nl; ++i) {
    int64_t K = 0;
    for (int32_t a : T.anc[i]) {
      K += h->rank_row[a];
      for (int64_t b : denrow[a]) K += h->size[h->den_col[b]];
    }
    b_nkb[i] = (int32_t)((K + KB - 1) / KB);
    b_off[i] = btot;
    btot += panel_chunks((int32_t)h->size[T.leaves[i]], b_nkb[i]);
  }
  if ((rc = lp->B.alloc(btot))) return rc;
  {
    StagerT<uint4> st;
    if ((rc = st.init(lp->B.p, std::max<int64_t>(btot, 1), s))) return rc;
    std::vector<std::pair<const double*, int64_t>> colp;  // per column: start of the leaf's rows
    for (int32_t i = 0; i < nl && !st.err; ++i) {
      const int32_t lf = T.leaves[i];
      zoff[i] = (int64_t)zmap.size();
      colp.clear();
      for (int32_t a : T.anc[i])
        if (h->rank_row[a] > 0)
          for (int32_t j = 0; j < h->rank_row[a]; ++j) {
            colp.push_back({h->U + 2 * (h->U_off[a] + (int64_t)j * h->size[a] + (h->off[lf] - h->off[a])), 0});
            zmap.push_back((int32_t)(yh_off[a] + j));
          }
      for (int32_t a : T.anc[i])
        for (int64_t b : denrow[a]) {
          const int32_t sg = h->den_col[b];
          for (int64_t j = 0; j < h->size[sg]; ++j) {
            colp.push_back({h->D + 2 * (h->D_off[b] + j * h->size[a] + (h->off[lf] - h->off[a])), 0});
            zmap.push_back((int32_t)(-1 - (h->off[sg] + j)));
          }
        }
      const int64_t K = (int64_t)colp.size();
      while ((int64_t)zmap.size() < zoff[i] + (int64_t)b_nkb[i] * KB) zmap.push_back(kZero);
      if ((rc = pack_panel<ST>(st, (int32_t)h->size[lf], b_nkb[i], [&](int32_t m, int32_t k) -> C {
             return k < K ? cget(colp[k].first, m) : C(0.0, 0.0);
           })))
        return rc;
    }
    if (btot > 0 && (rc = st.finish())) return rc;
  }
  for (int32_t m : zmap)
    if (m >= nyh || (m < 0 && m != kZero && -1 - (int64_t)m >= h->n)) return fail(UHM_EINVAL, "layout: gather index");
  if ((rc = lp->b_off.upload(b_off, s)) || (rc = lp->b_nkb.upload(b_nkb, s)) || (rc = lp->zoff.upload(zoff, s)) ||
      (rc = lp->zmap.upload(zmap, s)))
    return rc;
  UHM_HIP(hipStreamSynchronize(s));

  uhm_op_info& I = op->info;
  I.n = h->n;
  I.kind = 0;
  I.storage = ST;
  I.nleaves = nl;
  I.elem_bytes = ST == UHM_C64 ? 8 : 4;
  I.nadm = h->nadm;
  I.nden = h->nden;
  I.elems_forward = I.elems_backward = I.elems_coupling = I.elems_near = 0;
  for (int32_t c = 0; c < nc; ++c) {
    I.elems_forward += h->size[c] * h->rank_col[c];
    I.elems_backward += h->size[c] * h->rank_row[c];
  }
  for (int64_t b = 0; b < h->nadm; ++b) I.elems_coupling += (int64_t)h->rank_row[h->adm_row[b]] * h->rank_col[h->adm_col[b]];
  for (int64_t b = 0; b < h->nden; ++b) I.elems_near += h->size[h->den_row[b]] * h->size[h->den_col[b]];
  I.rank_space = nxh;
  I.device_bytes = (int64_t)(lp->F.bytes() + lp->S.bytes() + lp->B.bytes() + lp->zmap.bytes() + lp->colsrc.bytes());
  return UHM_OK;
}

template <int ST, int NT>
void launch_all(uhm_op* op, LowpOp* lp, const cf* x, int64_t ldx, cf* y, int64_t ldy, int r, int R, hipStream_t s) {
  const int nl = op->nleaves;
  const int64_t n = op->n;
  {
    ScopedTiming tm(op, s, K_LP_GATHER);
    hipLaunchKernelGGL(k_lp_gather, dim3((unsigned)((n * R + 255) / 256)), dim3(256), 0, s, x, ldx, r, R, op->perm.p, n,
                       lp->Xc.p);
  }
  if (lp->nxh > 0) {
    {
      ScopedTiming tm(op, s, K_LP_FORWARD);
      hipLaunchKernelGGL((k_lp_forward<ST, NT>), dim3(nl), dim3(64 * kLpWaves), 0, s, lp->F.p, lp->f_off.p, lp->f_M.p,
                         lp->f_nkb.p, op->leaf_pos.p, op->leaf_n.p, lp->poff.p, lp->Xc.p, R, lp->p.p);
    }
    {
      ScopedTiming tm(op, s, K_LP_REDUCE_FWD);
      hipLaunchKernelGGL(k_lp_reduce_segments, dim3((unsigned)((lp->nxh * R + 255) / 256)), dim3(256), 0, s, lp->p.p, R,
                         lp->poff.p, lp->out_seg.p, lp->seg_start.p, lp->seg_leaf0.p, lp->seg_nleaf.p, lp->seg_col.p,
                         lp->nxh, lp->xh.p);
    }
  }
  if (lp->nctiles > 0) {
    {
      ScopedTiming tm(op, s, K_LP_COUPLING);
      hipLaunchKernelGGL((k_lp_coupling<ST, NT>), dim3(lp->nctiles), dim3(64 * kLpWaves), 0, s, lp->S.p, lp->ctiles.p,
                         lp->colsrc.p, lp->xh.p, R, lp->part.p);
    }
    {
      ScopedTiming tm(op, s, K_LP_REDUCE_COUP);
      hipLaunchKernelGGL(k_lp_reduce_coupling, dim3((unsigned)((lp->nyh * R + 255) / 256)), dim3(256), 0, s, lp->part.p,
                         R, lp->yh_grp.p, lp->grp_start.p, lp->grp_t0.p, lp->grp_nt.p, lp->nyh, lp->yh.p);
    }
  }
  {
    ScopedTiming tm(op, s, K_LP_BACKWARD);
    hipLaunchKernelGGL((k_lp_backward<ST, NT>), dim3(nl), dim3(64 * kLpWaves), 0, s, lp->B.p, lp->b_off.p, lp->b_nkb.p,
                       lp->zoff.p, lp->zmap.p, op->leaf_pos.p, op->leaf_n.p, lp->yh.p, lp->Xc.p, R, lp->Yc.p);
  }
  {
    ScopedTiming tm(op, s, K_LP_SCATTER);
    hipLaunchKernelGGL(k_lp_scatter, dim3((unsigned)((n * r + 255) / 256)), dim3(256), 0, s, lp->Yc.p, r, R, op->perm.p,
                       n, y, ldy);
  }
}

template <int ST>
void launch_nt(uhm_op* op, LowpOp* lp, const cf* x, int64_t ldx, cf* y, int64_t ldy, int r, int R, hipStream_t s) {
  switch (R / 16) {
    case 1: launch_all<ST, 1>(op, lp, x, ldx, y, ldy, r, R, s); break;
    case 2: launch_all<ST, 2>(op, lp, x, ldx, y, ldy, r, R, s); break;
    case 3: launch_all<ST, 3>(op, lp, x, ldx, y, ldy, r, R, s); break;
    default: launch_all<ST, 4>(op, lp, x, ldx, y, ldy, r, R, s); break;
  }
}

int grow(LowpOp* lp, int64_t n, int R) {
  if (lp->wsR >= R) return UHM_OK;
  int rc;
  if ((rc = lp->Xc.alloc(n * R)) || (rc = lp->Yc.alloc(n * R)) || (rc = lp->p.alloc(std::max<int64_t>(1, lp->p_rows * R))) ||
      (rc = lp->xh.alloc(std::max<int64_t>(1, lp->nxh * R))) ||
      (rc = lp->part.alloc(std::max<int64_t>(1, (int64_t)lp->nctiles * 64 * R))) ||
      (rc = lp->yh.alloc(std::max<int64_t>(1, lp->nyh * R)))) {
    lp->wsR = 0;
    return rc;
  }
  lp->wsR = R;
  return UHM_OK;
}

}  // namespace

int lowp_upload(const uhm_host_operator* h, uhm_storage storage, hipStream_t s, const TreeInfo& T, uhm_op* op) {
  std::unique_ptr<LowpOp> lp(new (std::nothrow) LowpOp);
  if (!lp) return fail(UHM_ENOMEM, "host allocation");
  lp->storage = storage;
  lp->KB = storage == UHM_C64 ? Frag<UHM_C64>::KB : Frag<UHM_BF16PAIR>::KB;
  const int rc = storage == UHM_C64 ? lowp_upload_t<UHM_C64>(h, s, T, op, lp.get())
                                    : lowp_upload_t<UHM_BF16PAIR>(h, s, T, op, lp.get());
  if (rc) return rc;
  op->lp = lp.release();
  return UHM_OK;
}

int lowp_matvec(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, hipStream_t s) {
  LowpOp* lp = op->lp;
  if (!lp) return fail(UHM_EINVAL, "operator has no low-precision form");
  const cf* x = static_cast<const cf*>(X);
  cf* y = static_cast<cf*>(Y);
  for (int32_t c0 = 0; c0 < nrhs; c0 += kLpRmax) {
    const int r = std::min(kLpRmax, nrhs - c0);
    const int R = 16 * ((r + 15) / 16);
    int rc = grow(lp, op->n, std::max(R, lp->wsR));
    if (rc) return rc;
    if (lp->storage == UHM_C64)
      launch_nt<UHM_C64>(op, lp, x + (int64_t)c0 * ldx, ldx, y + (int64_t)c0 * ldy, ldy, r, R, s);
    else
      launch_nt<UHM_BF16PAIR>(op, lp, x + (int64_t)c0 * ldx, ldx, y + (int64_t)c0 * ldy, ldy, r, R, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(UHM_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return UHM_OK;
}

}  // namespace uhm_detail
