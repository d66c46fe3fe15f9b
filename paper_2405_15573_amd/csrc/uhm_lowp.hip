// Many-right-hand-side forms of the uniform H-matrix product on MFMA: complex64 storage
// (FP32 MFMA), (re, im) bfloat16 pairs (BF16 MFMA), both with FP32 accumulation, and
// complex128 storage (FP64 MFMA), 1 to 64 right-hand sides per pass.  The three stages of Algorithm 6 (section 4.4) become batched complex GEMMs:
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
// the only bf16 rounding is that of the stored operator.  In the bf16 form the vectors that
// feed a B operand (the gathered x, u_sigma, t_b, u_tau) are written split, once per
// product, by the kernels that produce them: each element is (re_hi, re_lo, im_hi, im_lo),
// 8 bytes, so staging a round copies bf16 parts instead of splitting FP32 values again in
// every tile that reads them.
//
// MFMA lane layouts (checked on gfx950):
//   v_mfma_f32_16x16x4_f32:  A lane l = A[l%16][l/16], B lane l = B[l/16][l%16]
//   v_mfma_f32_16x16x32_bf16: A lane l = A[l%16][8(l/16)+t], B lane l = B[8(l/16)+t][l%16]
//   both: accumulator register v of lane l = C[4(l/16)+v][l%16];
//   v_mfma_f64_16x16x4_f64: A, B as the f32 form, register v of lane l = C[l/16 + 4v][l%16].
// The k index inside one instruction may be any permutation shared by A and B; here lane
// group g = l/16 owns the k-values g*KPL .. g*KPL+KPL-1 of the k-block.
#include "uhm_internal.h"

#include <climits>
#include <complex>
#include <functional>
#include <map>
#include <cstring>

namespace uhm_detail {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
using cf = float2;

constexpr int kLpWaves = 4;
constexpr int kLpCoupK = 1024;      // coupling tile width in columns
constexpr int kFwdGroupRows = 256;  // rows of the largest forward panels
constexpr int kLpRmax = 64;         // right-hand sides per pass
constexpr int32_t kZero = INT_MIN;  // gather-map entry for a zero (padding) column

// ---- LDS images of the B operand for one round of RZ k-rows and R = 16 NT columns, sized
// for R so that passes with few right-hand sides leave room for more resident workgroups
template <int RZ, int NT>
struct LdsF32 {
  static constexpr int S = 16 * NT + 4;  // row stride (elements)
  cf z[RZ * S];
};
template <int RZ, int NT>
struct LdsF64 {
  static constexpr int S = 16 * NT + 4;
  cd z[RZ * S];
};
template <int RZ, int NT>
struct LdsBf16 {
  static constexpr int ZT = RZ + 8;  // plane row stride (per column j): 4 dwords past a multiple of 32
  alignas(16) __bf16 re_hi[16 * NT * ZT];
  alignas(16) __bf16 re_lo[16 * NT * ZT];
  alignas(16) __bf16 im_hi[16 * NT * ZT];
  alignas(16) __bf16 im_lo[16 * NT * ZT];
};

// k-rows per LDS round: the storage's base round rz, for R = 16 nt columns
constexpr int round_rows(int rz, int nt) { return rz; }

// ---- one lane's A chunk of a k-block: KPL complex values of its row
struct ChunkF32 {
  v4f re, im;
};
struct ChunkBf16 {
  v8bf re, im;
};
struct ChunkF64 {
  v4d re, im;
};

// ---- accumulators of a wave's 16 x 16 NT output tile
// Three-product form (complex64, complex128): p = sum ar br, q = sum ai bi,
// s = sum (ar + ai)(br + bi); Re = p - q, Im = s - p - q (Gauss's trick: three real
// products per complex multiply-add instead of four).
template <class A, int NT>
struct Acc3 {
  A p[NT], q[NT], s[NT];
  __device__ void zero() {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) p[nt] = q[nt] = s[nt] = A{0, 0, 0, 0};
  }
  __device__ auto re(int nt, int v) const { return p[nt][v] - q[nt][v]; }
  __device__ auto im(int nt, int v) const { return s[nt][v] - p[nt][v] - q[nt][v]; }
};
// Four-product form (bf16 pairs, where ar + ai would be rounded to bf16 again, and
// complex128, where a third accumulator costs occupancy at many columns).
template <class A, int NT>
struct Acc2 {
  A r[NT], i[NT];
  __device__ void zero() {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) r[nt] = i[nt] = A{0, 0, 0, 0};
  }
  __device__ auto re(int nt, int v) const { return r[nt][v]; }
  __device__ auto im(int nt, int v) const { return i[nt][v]; }
};

// A complex vector element split into bf16 parts: v ~ (rh + rl) + i (ih + il), each part the
// nearest bf16 (rl, il: of the FP32 remainder), 8 bytes like a complex64.
struct bfs4 {
  uint16_t rh, rl, ih, il;
};

// Storage traits.  CH: 16-byte words per lane chunk; RZ: k-rows per LDS round; KP: k-rows
// of one column that a thread stages together (one packed LDS store per plane; bf16 pairs
// take 8 where the round's slots allow, see kp_of);
// V: vector element; ACC: accumulator register tile; rows of an accumulator register:
// C64/BF16 lane (g, i) register v holds row 4g + v, C128 holds row g + 4v.
template <int ST>
struct Tr;
template <>
struct Tr<UHM_C64> {
  static constexpr int KB = 16, KPL = 4, CH = 2, RZ = 64, KP = 1;
  using V = cf;
  using VB = cf;  // vectors that feed a B operand
  using ACC = v4f;
  template <int NT>
  using ACCS = Acc3<v4f, NT>;
  template <int NT>
  using LDS = LdsF32<round_rows(RZ, NT), NT>;
  using CHUNK = ChunkF32;
  __device__ static int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Tr<UHM_BF16PAIR> {
  static constexpr int KB = 32, KPL = 8, CH = 2, RZ = 64, KP = 4;
  using V = cf;
  using VB = bfs4;
  using ACC = v4f;
  template <int NT>
  using ACCS = Acc2<v4f, NT>;
  template <int NT>
  using LDS = LdsBf16<round_rows(RZ, NT), NT>;
  using CHUNK = ChunkBf16;
  __device__ static int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Tr<UHM_C128_MULTI> {
  static constexpr int KB = 16, KPL = 4, CH = 4, RZ = 32, KP = 1;
  using V = cd;
  using VB = cd;
  using ACC = v4d;
  // four products at every NT: three accumulators per column tile would leave one wave per
  // SIMD at NT >= 3, and one scheme for all NT keeps a column's rounding independent of
  // how many columns share its pass
  template <int NT>
  using ACCS = Acc2<v4d, NT>;
  template <int NT>
  using LDS = LdsF64<round_rows(RZ, NT), NT>;
  using CHUNK = ChunkF64;
  __device__ static int row(int g, int v) { return g + 4 * v; }
};

template <class V>
__device__ __forceinline__ V vzero();
template <>
__device__ __forceinline__ cf vzero<cf>() { return make_float2(0.f, 0.f); }
template <>
__device__ __forceinline__ cd vzero<cd>() { return make_double2(0.0, 0.0); }
template <>
__device__ __forceinline__ bfs4 vzero<bfs4>() { return bfs4{0, 0, 0, 0}; }

// A V value (complex64 or complex128) as the B-operand element VB.
template <class VB>
__device__ __forceinline__ VB to_vb(cf v);
template <>
__device__ __forceinline__ cf to_vb<cf>(cf v) { return v; }
template <>
__device__ __forceinline__ bfs4 to_vb<bfs4>(cf v) {
  const __bf16 rh = (__bf16)v.x, ih = (__bf16)v.y;
  const __bf16 rl = (__bf16)(v.x - (float)rh), il = (__bf16)(v.y - (float)ih);
  return bfs4{__builtin_bit_cast(uint16_t, rh), __builtin_bit_cast(uint16_t, rl), __builtin_bit_cast(uint16_t, ih),
              __builtin_bit_cast(uint16_t, il)};
}
template <class VB>
__device__ __forceinline__ VB to_vb(cd v);
template <>
__device__ __forceinline__ cd to_vb<cd>(cd v) { return v; }

template <int ST, int NT>
using LdsOf = typename Tr<ST>::template LDS<NT>;

template <int RZ, int NT>
__device__ __forceinline__ void lds_put(LdsF32<RZ, NT>& L, int k, int j, cf v) { L.z[k * L.S + j] = v; }
template <int RZ, int NT>
__device__ __forceinline__ void lds_put(LdsF64<RZ, NT>& L, int k, int j, cd v) { L.z[k * L.S + j] = v; }
template <int RZ, int NT>
__device__ __forceinline__ void lds_put(LdsBf16<RZ, NT>& L, int k, int j, bfs4 v) {
  L.re_hi[j * L.ZT + k] = __builtin_bit_cast(__bf16, v.rh);
  L.re_lo[j * L.ZT + k] = __builtin_bit_cast(__bf16, v.rl);
  L.im_hi[j * L.ZT + k] = __builtin_bit_cast(__bf16, v.ih);
  L.im_lo[j * L.ZT + k] = __builtin_bit_cast(__bf16, v.il);
}
// Rows k0 .. k0 + 7 (k0 a multiple of 8) of column j: one 16-byte store per plane, the
// same bank pattern as the MFMA fragment reads (column stride 4 dwords past a multiple of
// 32, so 8 consecutive columns cover the 32 banks once).
template <int RZ, int NT>
__device__ __forceinline__ void lds_put8(LdsBf16<RZ, NT>& L, int k0, int j, const bfs4* v) {
  const int o = j * L.ZT + k0;
  auto pack = [&](auto part) {
    uint32_t w[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) w[t] = (uint32_t)part(v[2 * t]) | ((uint32_t)part(v[2 * t + 1]) << 16);
    return make_uint4(w[0], w[1], w[2], w[3]);
  };
  *reinterpret_cast<uint4*>(&L.re_hi[o]) = pack([](const bfs4& e) { return e.rh; });
  *reinterpret_cast<uint4*>(&L.re_lo[o]) = pack([](const bfs4& e) { return e.rl; });
  *reinterpret_cast<uint4*>(&L.im_hi[o]) = pack([](const bfs4& e) { return e.ih; });
  *reinterpret_cast<uint4*>(&L.im_lo[o]) = pack([](const bfs4& e) { return e.il; });
}
// Rows k0 .. k0 + 3 (k0 a multiple of 4) of column j: one 8-byte store per plane.  Columns
// 8 apart share banks here (2-way conflicts), so this serves only rounds whose slots do not
// come in groups of 8.
template <int RZ, int NT>
__device__ __forceinline__ void lds_put4(LdsBf16<RZ, NT>& L, int k0, int j, const bfs4* v) {
  const int o = j * L.ZT + k0;
  *reinterpret_cast<uint2*>(&L.re_hi[o]) =
      make_uint2((uint32_t)v[0].rh | ((uint32_t)v[1].rh << 16), (uint32_t)v[2].rh | ((uint32_t)v[3].rh << 16));
  *reinterpret_cast<uint2*>(&L.re_lo[o]) =
      make_uint2((uint32_t)v[0].rl | ((uint32_t)v[1].rl << 16), (uint32_t)v[2].rl | ((uint32_t)v[3].rl << 16));
  *reinterpret_cast<uint2*>(&L.im_hi[o]) =
      make_uint2((uint32_t)v[0].ih | ((uint32_t)v[1].ih << 16), (uint32_t)v[2].ih | ((uint32_t)v[3].ih << 16));
  *reinterpret_cast<uint2*>(&L.im_lo[o]) =
      make_uint2((uint32_t)v[0].il | ((uint32_t)v[1].il << 16), (uint32_t)v[2].il | ((uint32_t)v[3].il << 16));
}

__device__ __forceinline__ void load_chunk(const uint4* p, bool act, ChunkF32& c) {
  uint4 a = make_uint4(0, 0, 0, 0), b = a;
  if (act) {
    a = p[0];
    b = p[1];
  }
  c.re = __builtin_bit_cast(v4f, a);
  c.im = __builtin_bit_cast(v4f, b);
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
__device__ __forceinline__ void load_chunk(const uint4* p, bool act, ChunkF64& c) {
  uint4 a0 = make_uint4(0, 0, 0, 0), a1 = a0, b0 = a0, b1 = a0;
  if (act) {
    a0 = p[0];
    a1 = p[1];
    b0 = p[2];
    b1 = p[3];
  }
  const double2 r0 = __builtin_bit_cast(double2, a0), r1 = __builtin_bit_cast(double2, a1);
  const double2 i0 = __builtin_bit_cast(double2, b0), i1 = __builtin_bit_cast(double2, b1);
  c.re = v4d{r0.x, r0.y, r1.x, r1.y};
  c.im = v4d{i0.x, i0.y, i1.x, i1.y};
}

// acc += A_chunk (16 rows x one k-block) * B (k-block rows kk0.. of the LDS round).
template <int NT, int RZ>
__device__ __forceinline__ void mma_block(const ChunkF32& a, const LdsF32<RZ, NT>& L, int kk0, int g, int i,
                                          Acc3<v4f, NT>& c) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = kk0 + g * 4 + t;
    const float ar = a.re[t], ai = a.im[t], as = ar + ai;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const cf b = L.z[k * L.S + nt * 16 + i];
      c.p[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, b.x, c.p[nt], 0, 0, 0);
      c.q[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, b.y, c.q[nt], 0, 0, 0);
      c.s[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, b.x + b.y, c.s[nt], 0, 0, 0);
    }
  }
}

template <int NT, int RZ>
__device__ __forceinline__ void mma_block(const ChunkF64& a, const LdsF64<RZ, NT>& L, int kk0, int g, int i,
                                          Acc2<v4d, NT>& c) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = kk0 + g * 4 + t;
    const double ar = a.re[t], ai = a.im[t], nai = -a.im[t];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const cd b = L.z[k * L.S + nt * 16 + i];
      c.r[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b.x, c.r[nt], 0, 0, 0);
      c.r[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai, b.y, c.r[nt], 0, 0, 0);
      c.i[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, b.y, c.i[nt], 0, 0, 0);
      c.i[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, b.x, c.i[nt], 0, 0, 0);
    }
  }
}

template <int NT, int RZ>
__device__ __forceinline__ void mma_block(const ChunkBf16& a, const LdsBf16<RZ, NT>& L, int kk0, int g, int i,
                                          Acc2<v4f, NT>& c) {
  uint4 neg = __builtin_bit_cast(uint4, a.im);
  neg.x ^= 0x80008000u;
  neg.y ^= 0x80008000u;
  neg.z ^= 0x80008000u;
  neg.w ^= 0x80008000u;
  const v8bf nai = __builtin_bit_cast(v8bf, neg);
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    const int o = (nt * 16 + i) * L.ZT + kk0 + g * 8;
    const v8bf brh = *reinterpret_cast<const v8bf*>(&L.re_hi[o]);
    const v8bf brl = *reinterpret_cast<const v8bf*>(&L.re_lo[o]);
    const v8bf bih = *reinterpret_cast<const v8bf*>(&L.im_hi[o]);
    const v8bf bil = *reinterpret_cast<const v8bf*>(&L.im_lo[o]);
    c.r[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, brh, c.r[nt], 0, 0, 0);
    c.r[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, brl, c.r[nt], 0, 0, 0);
    c.r[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai, bih, c.r[nt], 0, 0, 0);
    c.r[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai, bil, c.r[nt], 0, 0, 0);
    c.i[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, bih, c.i[nt], 0, 0, 0);
    c.i[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.re, bil, c.i[nt], 0, 0, 0);
    c.i[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.im, brh, c.i[nt], 0, 0, 0);
    c.i[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.im, brl, c.i[nt], 0, 0, 0);
  }
}

// Store the 16 x (16 NT) accumulator tile; register v of lane (g, i) holds row Tr::row(g, v).
// OV: V for partial sums and outputs, VB where the tile's values feed a later B operand.
template <int ST, int NT, class OV = typename Tr<ST>::V>
__device__ __forceinline__ void store_tile(OV* out, int64_t row0, int hm, int R, int g, int i,
                                           const typename Tr<ST>::template ACCS<NT>& c) {
  using V = typename Tr<ST>::V;
#pragma unroll
  for (int nt = 0; nt < NT; ++nt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = Tr<ST>::row(g, v);
      if (r < hm) {
        V o;
        o.x = c.re(nt, v);
        o.y = c.im(nt, v);
        out[(row0 + r) * R + nt * 16 + i] = to_vb<OV>(o);
      }
    }
}

// ---------------------------------------------------------------- stage bodies
// Each stage is a device function over one work item (an element block, a leaf or a
// coupling tile).  The single-operator kernels map blockIdx.x to the item; the batched
// kernels read (operator, item) from a work list and the operator's descriptor.

struct LpCoupTile {
  int64_t base;     // uint4 offset of the chunk panel (all its m-tiles)
  int64_t csrc;     // offset of the chunk's first column in the column-source map
  int32_t h;        // rows of the chunk (<= 64)
  int32_t nkb_all;  // k-blocks of the chunk panel (stride between its m-tiles)
  int32_t kb0;      // first k-block of this tile
  int32_t nkb;      // k-blocks in this tile
  int32_t part;     // partial-sum slot (rows part*64 ..)
};

// Everything a stage needs about one operator and its bound vectors.
struct LpDesc {
  const uint4 *F, *S, *B;
  const int64_t *f_off, *poff, *b_off, *zoff, *seg_start, *grp_start;
  const int32_t *f_M, *f_nkb, *f_pos, *f_n, *b_nkb, *zmap, *colsrc, *out_seg, *seg_pan0, *seg_npan, *seg_col;
  const int32_t *yh_grp, *grp_t0, *grp_nt, *leaf_pos, *leaf_n, *perm, *iperm;
  const LpCoupTile* ctiles;
  void *Xc, *Yc, *p, *xh, *part, *yh;
  const void* x;
  void* y;
  const cd* const* xcol;  // when set: column j of x / y is the complex128 vector xcol[j] / ycol[j]
  cd* const* ycol;
  int64_t ldx, ldy, n, nxh, nyh;
  int32_t r, R;
};

// The user-order vectors are column-major and the cluster-order images row-major, with rows
// permuted.  Both directions go through a tile of 64 consecutive user rows staged in LDS:
// each column's 64 user rows are one contiguous read or write, and each row's R values go
// to or come from its cluster position as one contiguous run.
constexpr int kGatherRows = 64;
constexpr int kGatherThreads = 256;

// Xc[iperm[i]][j] = x(i, j) for the tile's user rows i (zero for j >= r), as B-operand
// elements.  load(i, j) returns the user-order element.
template <class V, class VB, class Load>
__device__ __forceinline__ void gather_tile(int64_t i0, int64_t n, int r, int R, const int32_t* __restrict__ iperm,
                                            VB* __restrict__ Xc, V* lds, Load load) {
  const int S = R + 1;
  for (int e = threadIdx.x; e < kGatherRows * R; e += kGatherThreads) {
    const int j = e / kGatherRows, il = e - j * kGatherRows;
    const int64_t i = i0 + il;
    lds[il * S + j] = (i < n && j < r) ? load(i, j) : vzero<V>();
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kGatherRows * R; e += kGatherThreads) {
    const int il = e / R, j = e - il * R;
    const int64_t i = i0 + il;
    if (i < n) Xc[(int64_t)iperm[i] * R + j] = to_vb<VB>(lds[il * S + j]);
  }
}

// y(i, j) = Yc[iperm[i]][j] for the tile's user rows i and j < r; store(i, j, v) writes it.
template <class V, class Store>
__device__ __forceinline__ void scatter_tile(int64_t i0, int64_t n, int r, int R, const int32_t* __restrict__ iperm,
                                             const V* __restrict__ Yc, V* lds, Store store) {
  const int S = R + 1;
  for (int e = threadIdx.x; e < kGatherRows * r; e += kGatherThreads) {
    const int il = e / r, j = e - il * r;
    const int64_t i = i0 + il;
    if (i < n) lds[il * S + j] = Yc[(int64_t)iperm[i] * R + j];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kGatherRows * r; e += kGatherThreads) {
    const int j = e / kGatherRows, il = e - j * kGatherRows;
    const int64_t i = i0 + il;
    if (i < n) store(i, j, lds[il * S + j]);
  }
}

// One LDS round covers up to KBR k-blocks.  Its memory requests are issued in batches so a
// round waits on about two memory latencies, not one per element and per k-block: the
// gather indices of the B operand, then the A chunks of all its k-blocks, then the B values.
// Every load of a batch is issued unconditionally from an address that is always in bounds
// (out-of-range slots re-read a valid one) and results are masked where they are used, so
// no load waits on a branch and the waits count only the batch they need.
// k-rows of one column that a thread stages together: the storage's KP, raised to 8 for
// bf16 pairs when the thread's PQ slots of a round come in whole groups of 8 (16-byte LDS
// stores instead of 8-byte ones, which conflict).
template <int ST, int NT>
constexpr int kp_of() {
  constexpr int pq = round_rows(Tr<ST>::RZ, NT) * 16 * NT / (64 * kLpWaves);
  return Tr<ST>::KP == 1 ? 1 : (pq % 8 == 0 ? 8 : Tr<ST>::KP);
}

template <int ST, int NT>
struct Round {
  using T_ = Tr<ST>;
  static constexpr int RZN = round_rows(T_::RZ, NT);
  static constexpr int KBR = RZN / T_::KB;                    // k-blocks per round
  static constexpr int PQ = RZN * 16 * NT / (64 * kLpWaves);  // B elements per thread
  static constexpr int KP = kp_of<ST, NT>();
  static_assert(PQ % KP == 0, "slots come in whole groups of KP rows");
  static_assert(T_::KB % KP == 0, "a k-block holds whole groups");
  typename T_::CHUNK a[KBR];
  typename T_::VB v[PQ];
  int32_t id[PQ];
  bool ok[PQ];
};

// A chunks of k-blocks kb .. kb+nkr-1 (nkr >= 1) of an m-tile with hm >= 1 valid rows.
// Lanes of rows i >= hm re-read row 0 and slots b >= nkr re-read k-block kb: those values
// only reach accumulator rows that are never stored, or no MFMA at all.
template <int ST, int NT>
__device__ __forceinline__ void round_issue_a(Round<ST, NT>& Q, const uint4* tile, int kb, int nkr, int hm, int g,
                                              int i) {
  using T_ = Tr<ST>;
  const int ii = i < hm ? i : 0;
#pragma unroll
  for (int b = 0; b < Round<ST, NT>::KBR; ++b) {
    const int kbb = kb + (b < nkr ? b : 0);
    load_chunk(tile + (int64_t)kbb * T_::CH * 4 * hm + T_::CH * (g * hm + ii), true, Q.a[b]);
  }
}

// Element (k, j) of the round that slot u of this thread stages: slots come in groups of
// KP consecutive k of one column; group g of thread t is q = t + g 256 with
// k = KP (q / R) + u % KP, j = q % R (R = 16 NT), so a wave's loads of one k are contiguous.
template <int ST, int NT>
__device__ __forceinline__ void slot_kj(int u, int& k, int& j) {
  constexpr int R = 16 * NT, KP = kp_of<ST, NT>();
  const int q = threadIdx.x + (u / KP) * 64 * kLpWaves;
  k = KP * (q / R) + u % KP;
  j = q % R;
}

// Raw gather indices of the round's B elements; slots with k >= nk re-read k = nk - 1.
template <int ST, int NT, class Idx>
__device__ __forceinline__ void round_indices(Round<ST, NT>& Q, int nk, Idx idx) {
#pragma unroll
  for (int u = 0; u < Round<ST, NT>::PQ; ++u) {
    int k, j;
    slot_kj<ST, NT>(u, k, j);
    Q.id[u] = idx(min(k, nk - 1));
  }
}
// B values: src(index, j, ok) returns the element's address when ok, else any valid address.
template <int ST, int NT, class Src>
__device__ __forceinline__ void round_values(Round<ST, NT>& Q, int nk, Src src) {
#pragma unroll
  for (int u = 0; u < Round<ST, NT>::PQ; ++u) {
    int k, j;
    slot_kj<ST, NT>(u, k, j);
    Q.ok[u] = k < nk && Q.id[u] != kZero;
    Q.v[u] = *src(Q.id[u], j, Q.ok[u]);
  }
}
template <int ST, int NT>
__device__ __forceinline__ void round_commit(LdsOf<ST, NT>& L, const Round<ST, NT>& Q, int nk) {
  using V = typename Tr<ST>::VB;
  constexpr int KP = kp_of<ST, NT>();
#pragma unroll
  for (int u = 0; u < Round<ST, NT>::PQ; u += KP) {
    int k, j;
    slot_kj<ST, NT>(u, k, j);  // k is a multiple of KP and nk of KB, so the group is whole
    if (k < nk) {
      if constexpr (KP == 1) {
        lds_put(L, k, j, Q.ok[u] ? Q.v[u] : vzero<V>());
      } else {
        V w[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) w[t] = Q.ok[u + t] ? Q.v[u + t] : vzero<V>();
        if constexpr (KP == 8)
          lds_put8(L, k, j, w);
        else
          lds_put4(L, k, j, w);
      }
    }
  }
}
template <int ST, int NT>
__device__ __forceinline__ void round_mma(const Round<ST, NT>& Q, const LdsOf<ST, NT>& L, int nkr, int g, int i,
                                          typename Tr<ST>::template ACCS<NT>& c) {
#pragma unroll
  for (int b = 0; b < Round<ST, NT>::KBR; ++b)
    if (b < nkr) mma_block<NT, Round<ST, NT>::RZN>(Q.a[b], L, b * Tr<ST>::KB, g, i, c);
}

// P = F^* X for one forward panel (rows pan_pos .. pan_pos + pan_n - 1 of the cluster order).
template <int ST, int NT>
__device__ __forceinline__ void forward_body(LdsOf<ST, NT>& L, int pan, const uint4* __restrict__ F,
                                             const int64_t* __restrict__ f_off, const int32_t* __restrict__ f_M,
                                             const int32_t* __restrict__ f_nkb, const int32_t* __restrict__ pan_pos,
                                             const int32_t* __restrict__ pan_n, const int64_t* __restrict__ poff,
                                             const typename Tr<ST>::VB* __restrict__ Xc, int R,
                                             typename Tr<ST>::V* __restrict__ p) {
  using T_ = Tr<ST>;
  using Q_ = Round<ST, NT>;
  const int M = f_M[pan];
  if (M == 0) return;
  const int n = pan_n[pan], nkb = f_nkb[pan];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, i = lane & 15;
  const uint4* base = F + f_off[pan];
  const int nmt = (M + 15) >> 4;
  const typename T_::VB* xl = Xc + (int64_t)pan_pos[pan] * R;
  constexpr int KBR = Q_::KBR;
  // rows k < n of the leaf; padding rows read row 0 and are masked
  auto src = [&](int32_t k, int j, bool ok) { return xl + (ok ? (int64_t)k * R + j : 0); };
  auto row = [&](int k0) { return [=](int k) { return k0 + k < n ? k0 + k : kZero; }; };
  if (nkb <= KBR) {
    // the whole leaf fits one round: stage once, then sweep the m-tiles with the next
    // m-tile's A chunks in flight while the current one multiplies
    Q_ Q, Qn;
    int mt = w;
    round_indices<ST, NT>(Q, nkb * T_::KB, row(0));
    const int m0 = mt < nmt ? mt : 0;
    round_issue_a<ST, NT>(Q, base + (int64_t)m0 * nkb * T_::CH * 64, 0, nkb, min(16, M - 16 * m0), g, i);
    round_values<ST, NT>(Q, nkb * T_::KB, src);
    round_commit<ST, NT>(L, Q, nkb * T_::KB);
    __syncthreads();
    for (; mt < nmt; mt += kLpWaves) {
      const int hm = min(16, M - 16 * mt);
      const int mn = mt + kLpWaves < nmt ? mt + kLpWaves : mt;
      round_issue_a<ST, NT>(Qn, base + (int64_t)mn * nkb * T_::CH * 64, 0, nkb, min(16, M - 16 * mn), g, i);
      typename T_::template ACCS<NT> acc;
      acc.zero();
      round_mma<ST, NT>(Q, L, nkb, g, i, acc);
      store_tile<ST, NT>(p, poff[pan] + 16 * mt, hm, R, g, i, acc);
#pragma unroll
      for (int b = 0; b < KBR; ++b) Q.a[b] = Qn.a[b];
    }
  } else {
    // leaf rows in several rounds: m-tiles in groups of kLpWaves, restaged per group
    Q_ Q;
    for (int mt0 = 0; mt0 < nmt; mt0 += kLpWaves) {
      const int mt = mt0 + w;
      const int ma = mt < nmt ? mt : 0;
      const int hm = min(16, M - 16 * ma);
      const uint4* tile = base + (int64_t)ma * nkb * T_::CH * 64;
      typename T_::template ACCS<NT> acc;
      acc.zero();
      for (int kb = 0; kb < nkb; kb += KBR) {
        const int nkr = min(KBR, nkb - kb), nk = nkr * T_::KB;
        round_indices<ST, NT>(Q, nk, row(kb * T_::KB));
        round_issue_a<ST, NT>(Q, tile, kb, nkr, hm, g, i);
        round_values<ST, NT>(Q, nk, src);
        __syncthreads();
        round_commit<ST, NT>(L, Q, nk);
        __syncthreads();
        if (mt < nmt) round_mma<ST, NT>(Q, L, nkr, g, i, acc);
      }
      if (mt < nmt) store_tile<ST, NT>(p, poff[pan] + 16 * mt, hm, R, g, i, acc);
    }
  }
}

// xh[e][j] = sum over the panels of the segment of p[poff[panel] + col + e - start][j].
template <class V, class VB>
__device__ __forceinline__ void reduce_segments_body(int64_t q, const V* __restrict__ p, int R,
                                                     const int64_t* __restrict__ poff,
                                                     const int32_t* __restrict__ out_seg,
                                                     const int64_t* __restrict__ seg_start,
                                                     const int32_t* __restrict__ seg_pan0,
                                                     const int32_t* __restrict__ seg_npan,
                                                     const int32_t* __restrict__ seg_col, int64_t nout,
                                                     VB* __restrict__ xh) {
  if (q >= nout * R) return;
  const int64_t e = q / R;
  const int j = (int)(q - e * R);
  const int s = out_seg[e];
  const int col = seg_col[s] + (int)(e - seg_start[s]);
  const int l0 = seg_pan0[s], nl = seg_npan[s];
  V acc = vzero<V>();
  for (int qq = 0; qq < nl; ++qq) {
    const V v = p[(poff[l0 + qq] + col) * R + j];
    acc.x += v.x;
    acc.y += v.y;
  }
  xh[q] = to_vb<VB>(acc);
}

// Partial u_tau of one coupling tile (wave w = m-tile w of the chunk).
template <int ST, int NT, class OV = typename Tr<ST>::V>
__device__ __forceinline__ void coupling_body(LdsOf<ST, NT>& L, const LpCoupTile& T,
                                              const uint4* __restrict__ S, const int32_t* __restrict__ colsrc,
                                              const typename Tr<ST>::VB* __restrict__ xh, int R,
                                              OV* __restrict__ part) {
  using T_ = Tr<ST>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, i = lane & 15;
  const int nmt = (T.h + 15) >> 4;
  const int hm = min(16, T.h - 16 * w);
  typename T_::template ACCS<NT> acc;
  acc.zero();
  using Q_ = Round<ST, NT>;
  constexpr int KBR = Q_::KBR;
  // waves without an m-tile re-read m-tile 0 and skip the MFMAs
  const int hma = w < nmt ? hm : min(16, T.h);
  const uint4* tila = S + T.base + (int64_t)(w < nmt ? w : 0) * T.nkb_all * T_::CH * 64;
  // column c of the chunk reads xh row colsrc[c] (< 0: zero); masked slots read row 0
  auto src = [&](int32_t sc, int j, bool ok) { return xh + (ok ? (int64_t)sc * R + j : 0); };
  Q_ Q;
  for (int kb = 0; kb < T.nkb; kb += KBR) {
    const int nkr = min(KBR, T.nkb - kb), nk = nkr * T_::KB;
    const int32_t* cs = colsrc + T.csrc + (int64_t)(T.kb0 + kb) * T_::KB;
    round_indices<ST, NT>(Q, nk, [&](int k) {
      const int32_t sc = cs[k];
      return sc >= 0 ? sc : kZero;
    });
    round_issue_a<ST, NT>(Q, tila, T.kb0 + kb, nkr, hma, g, i);
    round_values<ST, NT>(Q, nk, src);
    __syncthreads();
    round_commit<ST, NT>(L, Q, nk);
    __syncthreads();
    if (w < nmt) round_mma<ST, NT>(Q, L, nkr, g, i, acc);
  }
  if (w < nmt) store_tile<ST, NT, OV>(part, (int64_t)T.part * 64 + 16 * w, hm, R, g, i, acc);
}

// Factor pass over all t rows of one column cluster sigma whose K = l_sigma fits one LDS
// round: the gathered u_sigma is staged once and each wave multiplies it by its m-tiles in
// turn, storing rows part * 64 + 16 mt .. of `out`.
template <int ST, int NT>
__device__ __forceinline__ void factor_body(LdsOf<ST, NT>& L, const LpCoupTile& T, const uint4* __restrict__ S,
                                            const int32_t* __restrict__ colsrc,
                                            const typename Tr<ST>::VB* __restrict__ xh, int R,
                                            typename Tr<ST>::VB* __restrict__ out) {
  using T_ = Tr<ST>;
  using Q_ = Round<ST, NT>;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, i = lane & 15;
  const int nmt = (T.h + 15) >> 4;
  const int nkr = T.nkb_all, nk = nkr * T_::KB;  // nkr <= KBR, checked at upload
  auto src = [&](int32_t sc, int j, bool ok) { return xh + (ok ? (int64_t)sc * R + j : 0); };
  const int32_t* cs = colsrc + T.csrc;
  Q_ Q;
  round_indices<ST, NT>(Q, nk, [&](int k) {
    const int32_t sc = cs[k];
    return sc >= 0 ? sc : kZero;
  });
  round_values<ST, NT>(Q, nk, src);
  round_commit<ST, NT>(L, Q, nk);
  __syncthreads();
  for (int mt = w; mt < nmt; mt += kLpWaves) {
    const int hm = min(16, T.h - 16 * mt);
    round_issue_a<ST, NT>(Q, S + T.base + (int64_t)mt * T.nkb_all * T_::CH * 64, 0, nkr, hm, g, i);
    typename T_::template ACCS<NT> acc;
    acc.zero();
    round_mma<ST, NT>(Q, L, nkr, g, i, acc);
    store_tile<ST, NT, typename Tr<ST>::VB>(out, (int64_t)T.part * 64 + 16 * mt, hm, R, g, i, acc);
  }
}

template <class V, class VB>
__device__ __forceinline__ void reduce_coupling_body(int64_t q, const V* __restrict__ part, int R,
                                                     const int32_t* __restrict__ yh_grp,
                                                     const int64_t* __restrict__ grp_start,
                                                     const int32_t* __restrict__ grp_t0,
                                                     const int32_t* __restrict__ grp_nt, int64_t nout,
                                                     VB* __restrict__ yh) {
  if (q >= nout * R) return;
  const int64_t e = q / R;
  const int j = (int)(q - e * R);
  const int gi = yh_grp[e];
  const int r = (int)(e - grp_start[gi]);
  const int t0 = grp_t0[gi], nt = grp_nt[gi];
  V acc = vzero<V>();
  for (int tt = 0; tt < nt; ++tt) {
    const V v = part[((int64_t)(t0 + tt) * 64 + r) * R + j];
    acc.x += v.x;
    acc.y += v.y;
  }
  yh[q] = to_vb<VB>(acc);
}

// Y_lambda = B_lambda Z_lambda for one leaf; Z gathered from yh (index >= 0), from the
// cluster-ordered input (index = -1 - position) or zero (kZero).
template <int ST, int NT>
__device__ __forceinline__ void backward_body(LdsOf<ST, NT>& L, int leaf, const uint4* __restrict__ B,
                                              const int64_t* __restrict__ b_off, const int32_t* __restrict__ b_nkb,
                                              const int64_t* __restrict__ zoff, const int32_t* __restrict__ zmap,
                                              const int32_t* __restrict__ leaf_pos, const int32_t* __restrict__ leaf_n,
                                              const typename Tr<ST>::VB* __restrict__ yh,
                                              const typename Tr<ST>::VB* __restrict__ Xc, int R,
                                              typename Tr<ST>::V* __restrict__ Yc) {
  using T_ = Tr<ST>;
  const int n = leaf_n[leaf], nkb = b_nkb[leaf];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, g = lane >> 4, i = lane & 15;
  const int nmt = (n + 15) >> 4;
  const int hm = min(16, n - 16 * w);
  const int32_t* zm = zmap + zoff[leaf];
  typename T_::template ACCS<NT> acc;
  acc.zero();
  using Q_ = Round<ST, NT>;
  constexpr int KBR = Q_::KBR;
  const int hma = w < nmt ? hm : min(16, n);
  const uint4* tila = B + b_off[leaf] + (int64_t)(w < nmt ? w : 0) * nkb * T_::CH * 64;
  // map entry m >= 0: yh row m; m < 0 (not kZero): row -1 - m of the cluster-ordered input
  auto src = [&](int32_t m, int j, bool ok) {
    return ok ? (m >= 0 ? yh + (int64_t)m * R + j : Xc + (int64_t)(-1 - m) * R + j) : Xc;
  };
  Q_ Q;
  for (int kb = 0; kb < nkb; kb += KBR) {
    const int nkr = min(KBR, nkb - kb), nk = nkr * T_::KB;
    const int32_t* zk = zm + kb * T_::KB;
    round_indices<ST, NT>(Q, nk, [&](int k) { return zk[k]; });
    round_issue_a<ST, NT>(Q, tila, kb, nkr, hma, g, i);
    round_values<ST, NT>(Q, nk, src);
    __syncthreads();
    round_commit<ST, NT>(L, Q, nk);
    __syncthreads();
    if (w < nmt) round_mma<ST, NT>(Q, L, nkr, g, i, acc);
  }
  if (w < nmt) store_tile<ST, NT>(Yc, (int64_t)leaf_pos[leaf] + 16 * w, hm, R, g, i, acc);
}

// ---------------------------------------------------------------- single-operator kernels

template <int ST>
__global__ __launch_bounds__(kGatherThreads) void k_lp_gather(const typename Tr<ST>::V* __restrict__ x, int64_t ldx,
                                                              int r, int R, const int32_t* __restrict__ iperm,
                                                              int64_t n, typename Tr<ST>::VB* __restrict__ Xc) {
  using V = typename Tr<ST>::V;
  __shared__ V lds[kGatherRows * (kLpRmax + 1)];
  gather_tile((int64_t)blockIdx.x * kGatherRows, n, r, R, iperm, Xc, lds,
              [&](int64_t i, int j) { return x[i + (int64_t)j * ldx]; });
}

template <class V>
__global__ __launch_bounds__(kGatherThreads) void k_lp_scatter(const V* __restrict__ Yc, int r, int R,
                                                               const int32_t* __restrict__ iperm, int64_t n,
                                                               V* __restrict__ y, int64_t ldy) {
  __shared__ V lds[kGatherRows * (kLpRmax + 1)];
  scatter_tile((int64_t)blockIdx.x * kGatherRows, n, r, R, iperm, Yc, lds,
               [&](int64_t i, int j, V v) { y[i + (int64_t)j * ldy] = v; });
}

// complex128 -> the storage's vector element, for inputs given as complex128 columns
template <class V>
__device__ __forceinline__ V from_c128(cd a);
template <>
__device__ __forceinline__ cf from_c128<cf>(cd a) { return make_float2((float)a.x, (float)a.y); }
template <>
__device__ __forceinline__ cd from_c128<cd>(cd a) { return a; }


template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lp_forward(
    const uint4* __restrict__ F, const int64_t* __restrict__ f_off, const int32_t* __restrict__ f_M,
    const int32_t* __restrict__ f_nkb, const int32_t* __restrict__ f_pos, const int32_t* __restrict__ f_n,
    const int64_t* __restrict__ poff, const typename Tr<ST>::VB* __restrict__ Xc, int R,
    typename Tr<ST>::V* __restrict__ p) {
  __shared__ LdsOf<ST, NT> L;
  forward_body<ST, NT>(L, blockIdx.x, F, f_off, f_M, f_nkb, f_pos, f_n, poff, Xc, R, p);
}

template <int ST>
__global__ __launch_bounds__(256) void k_lp_reduce_segments(const typename Tr<ST>::V* __restrict__ p, int R,
                                                            const int64_t* __restrict__ poff,
                                                            const int32_t* __restrict__ out_seg,
                                                            const int64_t* __restrict__ seg_start,
                                                            const int32_t* __restrict__ seg_pan0,
                                                            const int32_t* __restrict__ seg_npan,
                                                            const int32_t* __restrict__ seg_col, int64_t nout,
                                                            typename Tr<ST>::VB* __restrict__ xh) {
  reduce_segments_body((int64_t)blockIdx.x * 256 + threadIdx.x, p, R, poff, out_seg, seg_start, seg_pan0, seg_npan,
                       seg_col, nout, xh);
}

// OV: the partial-sum element V, or VB for the factored first pass, whose tiles are the t_b
// rows of the coupling source vector
template <int ST, int NT, class OV>
__global__ __launch_bounds__(64 * kLpWaves) void k_lp_coupling(const uint4* __restrict__ S,
                                                               const LpCoupTile* __restrict__ tiles,
                                                               const int32_t* __restrict__ colsrc,
                                                               const typename Tr<ST>::VB* __restrict__ xh, int R,
                                                               OV* __restrict__ part) {
  __shared__ LdsOf<ST, NT> L;
  const LpCoupTile T = tiles[blockIdx.x];
  coupling_body<ST, NT, OV>(L, T, S, colsrc, xh, R, part);
}

template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lp_factor(const uint4* __restrict__ S,
                                                             const LpCoupTile* __restrict__ tiles,
                                                             const int32_t* __restrict__ colsrc,
                                                             const typename Tr<ST>::VB* __restrict__ xh, int R,
                                                             typename Tr<ST>::VB* __restrict__ out) {
  __shared__ LdsOf<ST, NT> L;
  const LpCoupTile T = tiles[blockIdx.x];
  factor_body<ST, NT>(L, T, S, colsrc, xh, R, out);
}

template <int ST>
__global__ __launch_bounds__(256) void k_lp_reduce_coupling(const typename Tr<ST>::V* __restrict__ part, int R,
                                                            const int32_t* __restrict__ yh_grp,
                                                            const int64_t* __restrict__ grp_start,
                                                            const int32_t* __restrict__ grp_t0,
                                                            const int32_t* __restrict__ grp_nt, int64_t nout,
                                                            typename Tr<ST>::VB* __restrict__ yh) {
  reduce_coupling_body((int64_t)blockIdx.x * 256 + threadIdx.x, part, R, yh_grp, grp_start, grp_t0, grp_nt, nout, yh);
}

template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lp_backward(
    const uint4* __restrict__ B, const int64_t* __restrict__ b_off, const int32_t* __restrict__ b_nkb,
    const int64_t* __restrict__ zoff, const int32_t* __restrict__ zmap, const int32_t* __restrict__ leaf_pos,
    const int32_t* __restrict__ leaf_n, const typename Tr<ST>::VB* __restrict__ yh,
    const typename Tr<ST>::VB* __restrict__ Xc, int R, typename Tr<ST>::V* __restrict__ Yc) {
  __shared__ LdsOf<ST, NT> L;
  backward_body<ST, NT>(L, blockIdx.x, B, b_off, b_nkb, zoff, zmap, leaf_pos, leaf_n, yh, Xc, R, Yc);
}

// ---------------------------------------------------------------- batched kernels
// work[b] = (operator, item): item is a 256-element block for the element-wise stages,
// a leaf for forward/backward, a coupling tile index (into the descriptor's tile array).

// work item: (operator, tile of kGatherRows user rows)
template <int ST>
__global__ __launch_bounds__(kGatherThreads) void k_lpb_gather(const LpDesc* __restrict__ D,
                                                               const int2* __restrict__ work) {
  using V = typename Tr<ST>::V;
  using VB = typename Tr<ST>::VB;
  __shared__ V lds[kGatherRows * (kLpRmax + 1)];
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  const int64_t i0 = (int64_t)wk.y * kGatherRows;
  if (d.xcol) {
    const cd* const* xc = d.xcol;
    gather_tile(i0, d.n, d.r, d.R, d.iperm, static_cast<VB*>(d.Xc), lds,
                [&](int64_t i, int j) { return from_c128<V>(xc[j][i]); });
  } else {
    const V* x = static_cast<const V*>(d.x);
    const int64_t ldx = d.ldx;
    gather_tile(i0, d.n, d.r, d.R, d.iperm, static_cast<VB*>(d.Xc), lds,
                [&](int64_t i, int j) { return x[i + (int64_t)j * ldx]; });
  }
}

template <class V>
__global__ __launch_bounds__(kGatherThreads) void k_lpb_scatter(const LpDesc* __restrict__ D,
                                                                const int2* __restrict__ work) {
  __shared__ V lds[kGatherRows * (kLpRmax + 1)];
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  const int64_t i0 = (int64_t)wk.y * kGatherRows;
  if (d.ycol) {
    cd* const* yc = d.ycol;
    scatter_tile(i0, d.n, d.r, d.R, d.iperm, static_cast<const V*>(d.Yc), lds,
                 [&](int64_t i, int j, V v) { yc[j][i] = make_double2((double)v.x, (double)v.y); });
  } else {
    V* y = static_cast<V*>(d.y);
    const int64_t ldy = d.ldy;
    scatter_tile(i0, d.n, d.r, d.R, d.iperm, static_cast<const V*>(d.Yc), lds,
                 [&](int64_t i, int j, V v) { y[i + (int64_t)j * ldy] = v; });
  }
}

template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lpb_forward(const LpDesc* __restrict__ D, const int2* __restrict__ work) {
  __shared__ LdsOf<ST, NT> L;
  using V = typename Tr<ST>::V;
  using VB = typename Tr<ST>::VB;
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  forward_body<ST, NT>(L, wk.y, d.F, d.f_off, d.f_M, d.f_nkb, d.f_pos, d.f_n, d.poff,
                       static_cast<const VB*>(d.Xc), d.R, static_cast<V*>(d.p));
}

template <int ST>
__global__ __launch_bounds__(256) void k_lpb_reduce_segments(const LpDesc* __restrict__ D, const int2* __restrict__ work) {
  using V = typename Tr<ST>::V;
  using VB = typename Tr<ST>::VB;
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  reduce_segments_body((int64_t)wk.y * 256 + threadIdx.x, static_cast<const V*>(d.p), d.R, d.poff, d.out_seg,
                       d.seg_start, d.seg_pan0, d.seg_npan, d.seg_col, d.nxh, static_cast<VB*>(d.xh));
}

// OV as in k_lp_coupling (VB for the factored first pass, whose descriptor's part points
// into the coupling source vector)
template <int ST, int NT, class OV>
__global__ __launch_bounds__(64 * kLpWaves) void k_lpb_coupling(const LpDesc* __restrict__ D, const int2* __restrict__ work) {
  __shared__ LdsOf<ST, NT> L;
  using VB = typename Tr<ST>::VB;
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  const LpCoupTile T = d.ctiles[wk.y];
  coupling_body<ST, NT, OV>(L, T, d.S, d.colsrc, static_cast<const VB*>(d.xh), d.R, static_cast<OV*>(d.part));
}

template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lpb_factor(const LpDesc* __restrict__ D, const int2* __restrict__ work) {
  __shared__ LdsOf<ST, NT> L;
  using VB = typename Tr<ST>::VB;
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  const LpCoupTile T = d.ctiles[wk.y];
  factor_body<ST, NT>(L, T, d.S, d.colsrc, static_cast<const VB*>(d.xh), d.R, static_cast<VB*>(d.part));
}

template <int ST>
__global__ __launch_bounds__(256) void k_lpb_reduce_coupling(const LpDesc* __restrict__ D, const int2* __restrict__ work) {
  using V = typename Tr<ST>::V;
  using VB = typename Tr<ST>::VB;
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  reduce_coupling_body((int64_t)wk.y * 256 + threadIdx.x, static_cast<const V*>(d.part), d.R, d.yh_grp, d.grp_start,
                       d.grp_t0, d.grp_nt, d.nyh, static_cast<VB*>(d.yh));
}

template <int ST, int NT>
__global__ __launch_bounds__(64 * kLpWaves) void k_lpb_backward(const LpDesc* __restrict__ D, const int2* __restrict__ work) {
  __shared__ LdsOf<ST, NT> L;
  using V = typename Tr<ST>::V;
  using VB = typename Tr<ST>::VB;
  const int2 wk = work[blockIdx.x];
  const LpDesc& d = D[wk.x];
  backward_body<ST, NT>(L, wk.y, d.B, d.b_off, d.b_nkb, d.zoff, d.zmap, d.leaf_pos, d.leaf_n,
                        static_cast<const VB*>(d.yh), static_cast<const VB*>(d.Xc), d.R, static_cast<V*>(d.Yc));
}

}  // namespace

// ---------------------------------------------------------------- host side

struct LowpOp {
  int storage = UHM_C64;
  int KB = 16;
  DevArray<uint4> F, S, B;
  DevArray<int64_t> f_off, poff, b_off, zoff, seg_start, grp_start;
  DevArray<int32_t> f_M, f_nkb, f_pos, f_n, b_nkb, zmap, colsrc, out_seg, seg_pan0, seg_npan, seg_col, yh_grp, grp_t0,
      grp_nt;
  int32_t npan = 0;  // forward panels
  DevArray<LpCoupTile> ctiles;
  int64_t p_rows = 0, nxh = 0, nyh = 0;
  int32_t nctiles = 0;
  // host copies for re-tiling the couplings (batched launches): one entry per row chunk
  struct Chunk {
    int64_t base, csrc;
    int32_t h, nkb_all;
    int32_t slot = -1;  // factor pass: 64-row slot of the output rows
  };
  std::vector<Chunk> chunks;
  // factored couplings (section 4.2): a first coupling pass whose rows are the t_b =
  // S_{Y,b}^* u_sigma of the factored blocks, grouped by column cluster sigma; one tile per
  // 64-row chunk (K = l_sigma), written straight to rows nxh .. nxh + ntf of the xh buffer
  // (each cluster's rows start on a multiple of 64), where the main pass reads them
  DevArray<uint4> ST;
  DevArray<int32_t> tcolsrc;
  DevArray<LpCoupTile> tctiles;  // clusters with l_sigma beyond one LDS round: 64-row chunks
  DevArray<LpCoupTile> tftiles;  // the others: one tile with all the cluster's t rows
  int32_t ntctiles = 0, ntftiles = 0;
  int64_t ntf = 0;
  std::vector<Chunk> tchunks;
  std::vector<int32_t> f_M_h, b_nkb_h, f_nkb_h, leaf_n_h;
  // workspace, sized for R columns
  int wsR = 0;
  DevArray<unsigned char> Xc, Yc, p, xh, part, yh;  // vector element: 8 or 16 bytes
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
  constexpr int KB = Tr<ST>::KB, KPL = Tr<ST>::KPL, CH = Tr<ST>::CH;
  std::complex<double> v[KPL];
  for (int32_t mt = 0; 16 * mt < M; ++mt) {
    const int32_t hm = std::min(16, M - 16 * mt);
    for (int32_t kb = 0; kb < nkb; ++kb) {
      uint4* dst = st.span((int64_t)CH * 4 * hm);
      for (int g = 0; g < 4; ++g)
        for (int32_t i = 0; i < hm; ++i) {
          for (int t = 0; t < KPL; ++t) v[t] = get(16 * mt + i, kb * KB + g * KPL + t);
          uint4* c = dst + CH * (g * hm + i);
          if (ST == UHM_C64) {
            float re[4], im[4];
            for (int t = 0; t < 4; ++t) {
              re[t] = (float)v[t].real();
              im[t] = (float)v[t].imag();
            }
            std::memcpy(&c[0], re, 16);
            std::memcpy(&c[1], im, 16);
          } else if (ST == UHM_BF16PAIR) {
            uint16_t re[8], im[8];
            for (int t = 0; t < 8; ++t) {
              re[t] = to_bf16((float)v[t].real());
              im[t] = to_bf16((float)v[t].imag());
            }
            std::memcpy(&c[0], re, 16);
            std::memcpy(&c[1], im, 16);
          } else {
            double re[4], im[4];
            for (int t = 0; t < 4; ++t) {
              re[t] = v[t].real();
              im[t] = v[t].imag();
            }
            std::memcpy(&c[0], re, 32);
            std::memcpy(&c[2], im, 32);
          }
        }
    }
  }
  return st.err;
}

template <int ST>
int64_t panel_chunks(int32_t M, int32_t nkb) {  // uint4 units
  return (int64_t)Tr<ST>::CH * 4 * M * nkb;
}

using C = std::complex<double>;

inline C cget(const double* a, int64_t idx) { return C(a[2 * idx], a[2 * idx + 1]); }

template <int ST>
int lowp_upload_t(const uhm_host_operator* h, hipStream_t s, const TreeInfo& T, uhm_op* op, LowpOp* lp, bool fact) {
  constexpr int KB = Tr<ST>::KB;
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

  // ---- forward panels.  Groups are the largest clusters of at most kFwdGroupRows rows;
  // they partition the index set.  The panel of a group g holds its rows of V_sigma for
  // every sigma containing g (root first); the panel of a leaf holds its rows of V_sigma for
  // the sigma strictly inside its group.  x_sigma is the sum of sigma's segment over the
  // panels that hold it, and the segment starts at the same column in each of them.  Group
  // panels cut the per-panel partial sums of the upper levels by up to kFwdGroupRows / leaf.
  std::vector<int32_t> gtop(nl);  // per leaf: index in anc of its group cluster
  for (int32_t i = 0; i < nl; ++i) {
    const std::vector<int32_t>& A = T.anc[i];
    int32_t q = (int32_t)A.size() - 1;
    while (q > 0 && h->size[A[q - 1]] <= kFwdGroupRows) --q;
    gtop[i] = q;
  }
  struct Pan {
    int32_t cl, leaf, a0, a1;  // rows of cluster cl; columns of anc[leaf][a0 .. a1)
  };
  std::vector<Pan> pans;
  for (int32_t i = 0; i < nl; ++i)  // group panels, in position order
    if (i == 0 || T.anc[i][gtop[i]] != T.anc[i - 1][gtop[i - 1]]) pans.push_back({T.anc[i][gtop[i]], i, 0, gtop[i] + 1});
  for (int32_t i = 0; i < nl; ++i)  // leaf panels: clusters strictly inside the group
    pans.push_back({T.leaves[i], i, gtop[i] + 1, (int32_t)T.anc[i].size()});
  std::vector<int64_t> f_off, poff;
  std::vector<int32_t> f_M, f_nkb, f_pos, f_n, seg_col_of(nc, -1), seg_pan0(nc, -1), seg_npan(nc, 0);
  int64_t ftot = 0, prow = 0;
  std::vector<Pan> kept;
  for (const Pan& P : pans) {
    int32_t Cn = 0;
    for (int32_t q = P.a0; q < P.a1; ++q) Cn += std::max(0, h->rank_col[T.anc[P.leaf][q]]);
    if (Cn == 0) continue;
    const int32_t pi = (int32_t)kept.size();
    Cn = 0;
    for (int32_t q = P.a0; q < P.a1; ++q) {
      const int32_t a = T.anc[P.leaf][q];
      if (h->rank_col[a] <= 0) continue;
      if (seg_col_of[a] < 0) seg_col_of[a] = Cn;
      if (seg_col_of[a] != Cn) return fail(UHM_EINVAL, "layout: forward segment column differs between panels");
      if (seg_pan0[a] < 0) seg_pan0[a] = pi;
      if (seg_pan0[a] + seg_npan[a] != pi) return fail(UHM_EINVAL, "layout: forward panels of a cluster not contiguous");
      ++seg_npan[a];
      Cn += h->rank_col[a];
    }
    kept.push_back(P);
    f_M.push_back(Cn);
    f_n.push_back((int32_t)h->size[P.cl]);
    f_pos.push_back((int32_t)h->off[P.cl]);
    f_nkb.push_back((int32_t)((h->size[P.cl] + KB - 1) / KB));
    f_off.push_back(ftot);
    poff.push_back(prow);
    ftot += panel_chunks<ST>(Cn, f_nkb.back());
    prow += Cn;
  }
  const int32_t npan = (int32_t)kept.size();
  if ((rc = lp->F.alloc(ftot))) return rc;
  if (ftot > 0) {
    StagerT<uint4> st;
    if ((rc = st.init(lp->F.p, ftot, s))) return rc;
    std::vector<const double*> colp;  // per panel column: start of the panel's rows in that basis column
    for (int32_t pi = 0; pi < npan && !st.err; ++pi) {
      const Pan& P = kept[pi];
      const int64_t n = h->size[P.cl];
      colp.clear();
      for (int32_t q = P.a0; q < P.a1; ++q) {
        const int32_t a = T.anc[P.leaf][q];
        for (int32_t j = 0; j < h->rank_col[a]; ++j)
          colp.push_back(h->V + 2 * (h->V_off[a] + (int64_t)j * h->size[a] + (h->off[P.cl] - h->off[a])));
      }
      if ((rc = pack_panel<ST>(st, f_M[pi], f_nkb[pi], [&](int32_t m, int32_t k) -> C {
             return k < n ? std::conj(cget(colp[m], k)) : C(0.0, 0.0);
           })))
        return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  if ((rc = lp->f_off.upload(f_off, s)) || (rc = lp->f_M.upload(f_M, s)) || (rc = lp->f_nkb.upload(f_nkb, s)) ||
      (rc = lp->f_pos.upload(f_pos, s)) || (rc = lp->f_n.upload(f_n, s)) || (rc = lp->poff.upload(poff, s)))
    return rc;
  lp->npan = npan;
  lp->f_M_h = f_M;
  lp->f_nkb_h = f_nkb;
  for (int32_t i = 0; i < nl; ++i) lp->leaf_n_h.push_back((int32_t)h->size[T.leaves[i]]);
  lp->p_rows = prow;
  // segments of x_sigma: sums over the panels that hold sigma
  {
    std::vector<int32_t> out_seg(nxh), p0, np, col;
    std::vector<int64_t> start;
    for (int32_t c = 0; c < nc; ++c) {
      if (h->rank_col[c] <= 0) continue;
      if (seg_pan0[c] < 0 || seg_npan[c] < 1 || seg_pan0[c] + seg_npan[c] > npan) return fail(UHM_EINVAL, "layout: segment");
      for (int32_t q = 0; q < seg_npan[c]; ++q)
        if (seg_col_of[c] < 0 || seg_col_of[c] + h->rank_col[c] > f_M[seg_pan0[c] + q])
          return fail(UHM_EINVAL, "layout: segment column");
      for (int32_t j = 0; j < h->rank_col[c]; ++j) out_seg[xh_off[c] + j] = (int32_t)start.size();
      start.push_back(xh_off[c]);
      p0.push_back(seg_pan0[c]);
      np.push_back(seg_npan[c]);
      col.push_back(seg_col_of[c]);
    }
    if ((rc = lp->out_seg.upload(out_seg, s)) || (rc = lp->seg_start.upload(start, s)) ||
        (rc = lp->seg_pan0.upload(p0, s)) || (rc = lp->seg_npan.upload(np, s)) || (rc = lp->seg_col.upload(col, s)))
      return rc;
  }
  lp->nxh = nxh;

  // ---- factored couplings: blocks with k_b (l_tau + l_sigma) < l_tau l_sigma keep their
  // factors; t_b = S_{Y,b}^* u_sigma is row t_off[b] .. of the t part of the xh buffer
  std::vector<char> fac(h->nadm, 0);
  std::vector<int64_t> t_off(h->nadm, -1);
  std::vector<std::vector<int64_t>> colfac(nc);
  int64_t ntf = 0;
  if (fact)
    for (int64_t b = 0; b < h->nadm; ++b) {
      const int64_t lt = h->rank_row[h->adm_row[b]], ls = h->rank_col[h->adm_col[b]], k = h->adm_rank[b];
      fac[b] = k * (lt + ls) < lt * ls;
      if (fac[b]) colfac[h->adm_col[b]].push_back(b);
    }
  for (int32_t c = 0; c < nc; ++c) {
    if (colfac[c].empty()) continue;
    ntf = (ntf + 63) & ~int64_t(63);  // the factor pass writes whole 64-row slots
    for (int64_t b : colfac[c]) {
      t_off[b] = ntf;
      ntf += h->adm_rank[b];
    }
  }
  if (nxh + ntf > INT32_MAX / kLpRmax) return fail(UHM_ENOTSUP, "rank space too large");
  {
    // first pass: for each column cluster sigma with factored blocks, the rows are the
    // columns of [S_{Y,b1} S_{Y,b2} ...] (conjugated), the columns are u_sigma
    std::vector<LpCoupTile> tt, tf;
    std::vector<int32_t> tcs;
    constexpr int KBR1 = Tr<ST>::RZ / KB;  // k-blocks of one LDS round
    struct TJob {
      int64_t m0, base;
      int32_t sg, hh, nkb;
    };
    std::vector<TJob> tj;
    int64_t tot = 0;
    for (int32_t c = 0; c < nc; ++c) {
      if (colfac[c].empty()) continue;
      const int32_t ls = h->rank_col[c];
      const int32_t nkb = (ls + KB - 1) / KB;
      const int64_t csrc = (int64_t)tcs.size();
      for (int32_t j = 0; j < ls; ++j) tcs.push_back((int32_t)(xh_off[c] + j));
      while ((int64_t)tcs.size() < csrc + (int64_t)nkb * KB) tcs.push_back(-1);
      int64_t M = 0;
      for (int64_t b : colfac[c]) M += h->adm_rank[b];
      const int64_t m0 = t_off[colfac[c][0]];
      if (nkb <= KBR1 && M <= INT32_MAX / 64) {  // u_sigma staged once for all its t rows
        tf.push_back({tot, csrc, (int32_t)M, nkb, 0, nkb, (int32_t)(m0 / 64)});
        tj.push_back({m0, tot, c, (int32_t)M, nkb});
        tot += panel_chunks<ST>((int32_t)M, nkb);
        continue;
      }
      for (int64_t r0 = 0; r0 < M; r0 += 64) {
        const int32_t hh = (int32_t)std::min<int64_t>(64, M - r0);
        const int32_t slot = (int32_t)((m0 + r0) / 64);
        tt.push_back({tot, csrc, hh, nkb, 0, nkb, slot});
        tj.push_back({m0 + r0, tot, c, hh, nkb});
        lp->tchunks.push_back({tot, csrc, hh, nkb, slot});
        tot += panel_chunks<ST>(hh, nkb);
      }
    }
    if ((rc = lp->ST.alloc(tot))) return rc;
    if (tot > 0) {
      std::vector<const double*> trow(ntf, nullptr);  // t row -> start of its S_{Y,b} column
      for (int32_t c = 0; c < nc; ++c)
        for (int64_t b : colfac[c])
          for (int32_t j = 0; j < h->adm_rank[b]; ++j)
            trow[t_off[b] + j] = h->SY + 2 * (h->SY_off[b] + (int64_t)j * h->rank_col[c]);
      StagerT<uint4> st;
      if ((rc = st.init(lp->ST.p, tot, s))) return rc;
      for (const TJob& J : tj) {
        if (st.err) break;
        const int32_t ls = h->rank_col[J.sg];
        if ((rc = pack_panel<ST>(st, J.hh, J.nkb, [&](int32_t m, int32_t k) -> C {
               return k < ls ? std::conj(cget(trow[J.m0 + m], k)) : C(0.0, 0.0);
             })))
          return rc;
      }
      if ((rc = st.finish())) return rc;
    }
    for (const LpCoupTile& Tt : tt)
      if (Tt.h < 1 || Tt.h > 64 || Tt.base < 0 || Tt.base + panel_chunks<ST>(Tt.h, Tt.nkb_all) > tot || Tt.kb0 < 0 ||
          Tt.nkb < 1 || Tt.kb0 + Tt.nkb > Tt.nkb_all || Tt.csrc + (int64_t)Tt.nkb_all * KB > (int64_t)tcs.size())
        return fail(UHM_EINVAL, "layout: factor tile");
    for (const LpCoupTile& Tt : tf)
      if (Tt.h < 1 || Tt.base < 0 || Tt.base + panel_chunks<ST>(Tt.h, Tt.nkb_all) > tot || Tt.nkb_all < 1 ||
          Tt.nkb_all > KBR1 || Tt.csrc + (int64_t)Tt.nkb_all * KB > (int64_t)tcs.size() || Tt.part < 0 ||
          (int64_t)Tt.part * 64 + Tt.h > ntf)
        return fail(UHM_EINVAL, "layout: factor tile");
    for (int32_t v : tcs)
      if (v >= nxh) return fail(UHM_EINVAL, "layout: factor column source");
    for (const LpCoupTile& Tt : tt)
      if (Tt.part < 0 || (int64_t)Tt.part * 64 + Tt.h > ntf) return fail(UHM_EINVAL, "layout: factor rows");
    if ((rc = lp->tctiles.upload(tt, s)) || (rc = lp->tftiles.upload(tf, s)) || (rc = lp->tcolsrc.upload(tcs, s)))
      return rc;
    lp->ntftiles = (int32_t)tf.size();
    lp->ntctiles = (int32_t)tt.size();
    lp->ntf = ntf;
  }

  // ---- couplings: row chunks of 64 rows, K padded to KB, tiles of kLpCoupK columns; a
  // factored block contributes S_{X,b} (columns reading t_b) in place of S_b (reading u_sigma)
  std::vector<std::vector<int64_t>> rowblk(nc);
  for (int64_t b = 0; b < h->nadm; ++b) rowblk[h->adm_row[b]].push_back(b);
  auto width = [&](int64_t b) -> int32_t { return fac[b] ? h->adm_rank[b] : h->rank_col[h->adm_col[b]]; };
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
    for (int64_t b : rowblk[t]) K += width(b);
    const int32_t nkb = (int32_t)((K + KB - 1) / KB);
    const int64_t csrc = (int64_t)colsrc.size();
    for (int64_t b : rowblk[t])
      for (int32_t j = 0; j < width(b); ++j)
        colsrc.push_back((int32_t)(fac[b] ? nxh + t_off[b] + j : xh_off[h->adm_col[b]] + j));
    while ((int64_t)colsrc.size() < csrc + (int64_t)nkb * KB) colsrc.push_back(-1);
    for (int32_t r0 = 0; r0 < lt; r0 += 64) {
      const int32_t hh = std::min(64, lt - r0);
      const int32_t gi = (int32_t)grp_start.size();
      grp_start.push_back(yh_off[t] + r0);
      grp_t0.push_back((int32_t)tiles.size());
      for (int32_t r = 0; r < hh; ++r) yh_grp[yh_off[t] + r0 + r] = gi;
      constexpr int KBT = kLpCoupK / KB;
      for (int32_t kb0 = 0; kb0 < nkb; kb0 += KBT)
        tiles.push_back({stot, csrc, hh, nkb, kb0, std::min(KBT, nkb - kb0), (int32_t)tiles.size()});
      grp_nt.push_back((int32_t)tiles.size() - grp_t0.back());
      jobs.push_back({t, r0, hh, stot, csrc, nkb});
      lp->chunks.push_back({stot, csrc, hh, nkb});
      stot += panel_chunks<ST>(hh, nkb);
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
        for (int32_t j = 0; j < width(b); ++j)
          colp.push_back({fac[b] ? h->SX + 2 * (h->SX_off[b] + (int64_t)j * lt + J.r0)
                                 : h->S + 2 * (h->S_off[b] + (int64_t)j * lt + J.r0),
                          lt});
      const int64_t K = (int64_t)colp.size();
      if ((rc = pack_panel<ST>(st, J.h, J.nkb, [&](int32_t m, int32_t k) -> C {
             return k < K ? cget(colp[k].first, m) : C(0.0, 0.0);
           })))
        return rc;
    }
    if ((rc = st.finish())) return rc;
  }
  for (const LpCoupTile& Tt : tiles) {
    if (Tt.h < 1 || Tt.h > 64 || Tt.base < 0 || Tt.base + panel_chunks<ST>(Tt.h, Tt.nkb_all) > stot ||
        Tt.kb0 < 0 || Tt.nkb < 1 || Tt.kb0 + Tt.nkb > Tt.nkb_all || Tt.csrc + (int64_t)Tt.nkb_all * KB > (int64_t)colsrc.size())
      return fail(UHM_EINVAL, "layout: coupling tile");
  }
  for (int32_t v : colsrc)
    if (v >= nxh + ntf) return fail(UHM_EINVAL, "layout: coupling column source");
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
    btot += panel_chunks<ST>((int32_t)h->size[T.leaves[i]], b_nkb[i]);
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
  lp->b_nkb_h = b_nkb;
  UHM_HIP(hipStreamSynchronize(s));

  uhm_op_info& I = op->info;
  I.n = h->n;
  I.kind = 0;
  I.storage = op->storage;
  I.nleaves = nl;
  I.elem_bytes = ST == UHM_C64 ? 8 : (ST == UHM_BF16PAIR ? 4 : 16);
  I.nadm = h->nadm;
  I.nden = h->nden;
  I.elems_forward = I.elems_backward = I.elems_coupling = I.elems_near = 0;
  for (int32_t c = 0; c < nc; ++c) {
    I.elems_forward += h->size[c] * h->rank_col[c];
    I.elems_backward += h->size[c] * h->rank_row[c];
  }
  I.elems_coupling_in = 0;
  for (int64_t b = 0; b < h->nadm; ++b) {
    const int64_t lt = h->rank_row[h->adm_row[b]], ls = h->rank_col[h->adm_col[b]];
    I.elems_coupling += fac[b] ? lt * h->adm_rank[b] : lt * ls;
    if (fac[b]) I.elems_coupling_in += ls * h->adm_rank[b];
  }
  for (int64_t b = 0; b < h->nden; ++b) I.elems_near += h->size[h->den_row[b]] * h->size[h->den_col[b]];
  I.rank_space = nxh;
  I.device_bytes = (int64_t)(lp->F.bytes() + lp->S.bytes() + lp->B.bytes() + lp->zmap.bytes() + lp->colsrc.bytes() +
                             lp->ST.bytes() + lp->tcolsrc.bytes());
  return UHM_OK;
}

template <int ST, int NT>
void launch_all(uhm_op* op, LowpOp* lp, const void* xv, int64_t ldx, void* yv, int64_t ldy, int r, int R, hipStream_t s) {
  using V = typename Tr<ST>::V;
  using VB = typename Tr<ST>::VB;
  static_assert(sizeof(VB) == sizeof(V), "workspace sized by the vector element");
  const V* x = static_cast<const V*>(xv);
  V* y = static_cast<V*>(yv);
  VB* Xc = reinterpret_cast<VB*>(lp->Xc.p);
  V* Yc = reinterpret_cast<V*>(lp->Yc.p);
  V* p = reinterpret_cast<V*>(lp->p.p);
  VB* xh = reinterpret_cast<VB*>(lp->xh.p);
  V* part = reinterpret_cast<V*>(lp->part.p);
  VB* yh = reinterpret_cast<VB*>(lp->yh.p);
  const int nl = op->nleaves;
  const int64_t n = op->n;
  {
    ScopedTiming tm(op, s, K_LP_GATHER);
    hipLaunchKernelGGL(k_lp_gather<ST>, dim3((unsigned)((n + kGatherRows - 1) / kGatherRows)), dim3(kGatherThreads), 0, s,
                       x, ldx, r, R, op->iperm.p, n, Xc);
  }
  if (lp->nxh > 0) {
    {
      ScopedTiming tm(op, s, K_LP_FORWARD);
      hipLaunchKernelGGL((k_lp_forward<ST, NT>), dim3(lp->npan), dim3(64 * kLpWaves), 0, s, lp->F.p, lp->f_off.p, lp->f_M.p,
                         lp->f_nkb.p, lp->f_pos.p, lp->f_n.p, lp->poff.p, Xc, R, p);
    }
    {
      ScopedTiming tm(op, s, K_LP_REDUCE_FWD);
      hipLaunchKernelGGL(k_lp_reduce_segments<ST>, dim3((unsigned)((lp->nxh * R + 255) / 256)), dim3(256), 0, s, p, R,
                         lp->poff.p, lp->out_seg.p, lp->seg_start.p, lp->seg_pan0.p, lp->seg_npan.p, lp->seg_col.p,
                         lp->nxh, xh);
    }
  }
  // factored couplings, first pass: t_b rows go straight to their slots after the nxh rows of u
  if (lp->ntftiles > 0) {
    ScopedTiming tm(op, s, K_LP_FACTOR_IN);
    hipLaunchKernelGGL((k_lp_factor<ST, NT>), dim3(lp->ntftiles), dim3(64 * kLpWaves), 0, s, lp->ST.p, lp->tftiles.p,
                       lp->tcolsrc.p, xh, R, xh + lp->nxh * R);
  }
  if (lp->ntctiles > 0) {
    ScopedTiming tm(op, s, K_LP_FACTOR_IN);
    hipLaunchKernelGGL((k_lp_coupling<ST, NT, VB>), dim3(lp->ntctiles), dim3(64 * kLpWaves), 0, s, lp->ST.p,
                       lp->tctiles.p, lp->tcolsrc.p, xh, R, xh + lp->nxh * R);
  }
  if (lp->nctiles > 0) {
    {
      ScopedTiming tm(op, s, K_LP_COUPLING);
      hipLaunchKernelGGL((k_lp_coupling<ST, NT, V>), dim3(lp->nctiles), dim3(64 * kLpWaves), 0, s, lp->S.p,
                         lp->ctiles.p, lp->colsrc.p, xh, R, part);
    }
    {
      ScopedTiming tm(op, s, K_LP_REDUCE_COUP);
      hipLaunchKernelGGL(k_lp_reduce_coupling<ST>, dim3((unsigned)((lp->nyh * R + 255) / 256)), dim3(256), 0, s, part, R,
                         lp->yh_grp.p, lp->grp_start.p, lp->grp_t0.p, lp->grp_nt.p, lp->nyh, yh);
    }
  }
  {
    ScopedTiming tm(op, s, K_LP_BACKWARD);
    hipLaunchKernelGGL((k_lp_backward<ST, NT>), dim3(nl), dim3(64 * kLpWaves), 0, s, lp->B.p, lp->b_off.p, lp->b_nkb.p,
                       lp->zoff.p, lp->zmap.p, op->leaf_pos.p, op->leaf_n.p, yh, Xc, R, Yc);
  }
  {
    ScopedTiming tm(op, s, K_LP_SCATTER);
    hipLaunchKernelGGL(k_lp_scatter<V>, dim3((unsigned)((n + kGatherRows - 1) / kGatherRows)), dim3(kGatherThreads), 0, s,
                       Yc, r, R, op->iperm.p, n,
                       y, ldy);
  }
}

template <int ST>
void launch_nt(uhm_op* op, LowpOp* lp, const void* x, int64_t ldx, void* y, int64_t ldy, int r, int R, hipStream_t s) {
  switch (R / 16) {
    case 1: launch_all<ST, 1>(op, lp, x, ldx, y, ldy, r, R, s); break;
    case 2: launch_all<ST, 2>(op, lp, x, ldx, y, ldy, r, R, s); break;
    case 3: launch_all<ST, 3>(op, lp, x, ldx, y, ldy, r, R, s); break;
    default: launch_all<ST, 4>(op, lp, x, ldx, y, ldy, r, R, s); break;
  }
}

int grow(LowpOp* lp, int64_t n, int R) {
  if (lp->wsR >= R) return UHM_OK;
  const int64_t e = lp->storage == UHM_C128_MULTI ? 16 : 8;
  int rc;
  if ((rc = lp->Xc.alloc(e * n * R)) || (rc = lp->Yc.alloc(e * n * R)) ||
      (rc = lp->p.alloc(e * std::max<int64_t>(1, lp->p_rows * R))) ||
      (rc = lp->xh.alloc(e * std::max<int64_t>(1, (lp->nxh + lp->ntf) * R))) ||
      (rc = lp->part.alloc(e * std::max<int64_t>(1, (int64_t)lp->nctiles * 64 * R))) ||
      (rc = lp->yh.alloc(e * std::max<int64_t>(1, lp->nyh * R)))) {
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
  // the factored forms run the kernels of their base form
  const bool fact =
      storage == UHM_C64_FACTORED || storage == UHM_BF16PAIR_FACTORED || storage == UHM_C128_MULTI_FACTORED;
  const int base = storage == UHM_C64_FACTORED        ? UHM_C64
                   : storage == UHM_BF16PAIR_FACTORED  ? UHM_BF16PAIR
                   : storage == UHM_C128_MULTI_FACTORED ? UHM_C128_MULTI
                                                        : storage;
  lp->storage = base;
  int rc;
  if (base == UHM_C64) {
    lp->KB = Tr<UHM_C64>::KB;
    rc = lowp_upload_t<UHM_C64>(h, s, T, op, lp.get(), fact);
  } else if (base == UHM_BF16PAIR) {
    lp->KB = Tr<UHM_BF16PAIR>::KB;
    rc = lowp_upload_t<UHM_BF16PAIR>(h, s, T, op, lp.get(), fact);
  } else {
    lp->KB = Tr<UHM_C128_MULTI>::KB;
    rc = lowp_upload_t<UHM_C128_MULTI>(h, s, T, op, lp.get(), fact);
  }
  if (rc) return rc;
  op->lp = lp.release();
  return UHM_OK;
}

int lowp_matvec(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, hipStream_t s) {
  LowpOp* lp = op->lp;
  if (!lp) return fail(UHM_EINVAL, "operator has no low-precision form");
  const int64_t e = lp->storage == UHM_C128_MULTI ? 16 : 8;
  const char* x = static_cast<const char*>(X);
  char* y = static_cast<char*>(Y);
  for (int32_t c0 = 0; c0 < nrhs; c0 += kLpRmax) {
    const int r = std::min(kLpRmax, nrhs - c0);
    const int R = 16 * ((r + 15) / 16);
    int rc = grow(lp, op->n, std::max(R, lp->wsR));
    if (rc) return rc;
    const void* xc = x + e * c0 * ldx;
    void* yc = y + e * c0 * ldy;
    if (lp->storage == UHM_C64)
      launch_nt<UHM_C64>(op, lp, xc, ldx, yc, ldy, r, R, s);
    else if (lp->storage == UHM_BF16PAIR)
      launch_nt<UHM_BF16PAIR>(op, lp, xc, ldx, yc, ldy, r, R, s);
    else
      launch_nt<UHM_C128_MULTI>(op, lp, xc, ldx, yc, ldy, r, R, s);
  }
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail(UHM_EHIP, std::string("kernel launch: ") + hipGetErrorString(he));
  return UHM_OK;
}

// ---------------------------------------------------------------- batched products

namespace {

struct BatchConfig {
  int32_t coup_cols = kLpCoupK;  // coupling tile width in columns
  int32_t order = 0;             // 0 operator-major, 1 cost-descending, 2 round-robin over cost buckets
};

// Candidate schedules the tuner times; winners are cached per batch signature.
const int32_t kTileWidths[] = {256, 512, 1024, 2048};
std::map<std::string, BatchConfig>& tune_cache() {
  static std::map<std::string, BatchConfig> m;
  return m;
}

struct BatchOp {
  uhm_op* op;
  const void* x;
  void* y;
  int64_t ldx, ldy;
  int32_t r;
  DevArray<unsigned char> Xc, Yc, p, xh, part, yh;
  DevArray<LpCoupTile> tiles;
  DevArray<int32_t> grp_t0, grp_nt;
  int32_t ntiles = 0;
  int64_t part_cap = 0;  // partial-sum slots allocated (tiles * 64 * R elements)
};

}  // namespace

struct LowpBatch {
  int storage = UHM_C64;
  int R = 16;
  std::vector<std::unique_ptr<BatchOp>> ops;
  BatchConfig cfg;
  bool configured = false;
  DevArray<LpDesc> desc;
  DevArray<int2> w_gather, w_forward, w_rseg, w_ffac, w_fcoup, w_coup, w_rcoup, w_backward, w_scatter;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string signature;
  ~LowpBatch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

namespace {

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Order a stage's work items: 0 keeps operator-major order, 1 sorts by cost (largest
// first), 2 deals items round-robin over cost buckets (powers of two), largest bucket first.
void order_work(std::vector<int2>& w, const std::vector<int64_t>& cost, int order) {
  if (order == 0 || w.size() < 2) return;
  std::vector<size_t> idx(w.size());
  for (size_t k = 0; k < idx.size(); ++k) idx[k] = k;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<int2> out;
  out.reserve(w.size());
  if (order == 1) {
    for (size_t k : idx) out.push_back(w[k]);
  } else {
    std::map<int, std::vector<size_t>, std::greater<int>> buckets;
    for (size_t k : idx) {
      int bkt = 0;
      for (int64_t c = cost[k]; c > 1; c >>= 1) ++bkt;
      buckets[bkt].push_back(k);
    }
    std::vector<std::pair<std::vector<size_t>*, size_t>> cur;
    for (auto& kv : buckets) cur.push_back({&kv.second, 0});
    bool any = true;
    while (any) {
      any = false;
      for (auto& c : cur)
        if (c.second < c.first->size()) {
          out.push_back(w[(*c.first)[c.second++]]);
          any = true;
        }
    }
  }
  w.swap(out);
}

// The operator's part of a batch descriptor: its panels, maps and tables.
LpDesc desc_of(uhm_op* op) {
  const LowpOp* lp = op->lp;
  LpDesc d{};
  d.F = lp->F.p;
  d.S = lp->S.p;
  d.B = lp->B.p;
  d.f_off = lp->f_off.p;
  d.poff = lp->poff.p;
  d.b_off = lp->b_off.p;
  d.zoff = lp->zoff.p;
  d.seg_start = lp->seg_start.p;
  d.grp_start = lp->grp_start.p;
  d.f_M = lp->f_M.p;
  d.f_nkb = lp->f_nkb.p;
  d.b_nkb = lp->b_nkb.p;
  d.zmap = lp->zmap.p;
  d.colsrc = lp->colsrc.p;
  d.out_seg = lp->out_seg.p;
  d.seg_pan0 = lp->seg_pan0.p;
  d.seg_npan = lp->seg_npan.p;
  d.f_pos = lp->f_pos.p;
  d.f_n = lp->f_n.p;
  d.seg_col = lp->seg_col.p;
  d.yh_grp = lp->yh_grp.p;
  d.leaf_pos = op->leaf_pos.p;
  d.leaf_n = op->leaf_n.p;
  d.perm = op->perm.p;
  d.iperm = op->iperm.p;
  d.n = op->n;
  d.nxh = lp->nxh;
  d.nyh = lp->nyh;
  return d;
}

// The descriptor of an operator's factored-coupling first pass, from the descriptor d of its
// main passes: the coupling stage reads the t-rows panel and writes its tiles (one per
// 64-row slot) straight into rows nxh .. of xh.
LpDesc factor_desc(const LowpOp* lp, const LpDesc& d, const LpCoupTile* tiles, int64_t ebytes) {
  LpDesc f = d;
  f.S = lp->ST.p;
  f.colsrc = lp->tcolsrc.p;
  f.ctiles = tiles;
  f.part = static_cast<unsigned char*>(d.xh) + ebytes * lp->nxh * d.R;
  return f;
}

int configure(LowpBatch* B, const BatchConfig& cfg, hipStream_t s) {
  const int KB = B->ops[0]->op->lp->KB;
  const int64_t e = B->storage == UHM_C128_MULTI ? 16 : 8;
  const int R = B->R;
  std::vector<LpDesc> descs, fdescs;
  std::vector<int2> wg, wf, wrs, wff, wfc, wc, wrc, wb, wsc;
  std::vector<int64_t> cf_, cfc_, cc_, cb_;
  const int32_t nops = (int32_t)B->ops.size();
  int rc;
  for (size_t k = 0; k < B->ops.size(); ++k) {
    BatchOp& bo = *B->ops[k];
    uhm_op* op = bo.op;
    LowpOp* lp = op->lp;
    // coupling tiles of width cfg.coup_cols over the operator's row chunks
    std::vector<LpCoupTile> tiles;
    std::vector<int32_t> t0, nt;
    const int32_t kbt = std::max(1, cfg.coup_cols / KB);
    for (const LowpOp::Chunk& c : lp->chunks) {
      t0.push_back((int32_t)tiles.size());
      for (int32_t kb0 = 0; kb0 < c.nkb_all; kb0 += kbt)
        tiles.push_back({c.base, c.csrc, c.h, c.nkb_all, kb0, std::min(kbt, c.nkb_all - kb0), (int32_t)tiles.size()});
      nt.push_back((int32_t)tiles.size() - t0.back());
    }
    if ((rc = bo.tiles.upload(tiles, s)) || (rc = bo.grp_t0.upload(t0, s)) || (rc = bo.grp_nt.upload(nt, s))) return rc;
    bo.ntiles = (int32_t)tiles.size();
    const int64_t need = std::max<int64_t>(1, (int64_t)bo.ntiles * 64 * R);
    if (bo.part_cap < need) {
      if ((rc = bo.part.alloc(e * need))) return rc;
      bo.part_cap = need;
    }
    LpDesc d = desc_of(op);
    d.grp_t0 = bo.grp_t0.p;
    d.grp_nt = bo.grp_nt.p;
    d.ctiles = bo.tiles.p;
    d.Xc = bo.Xc.p;
    d.Yc = bo.Yc.p;
    d.p = bo.p.p;
    d.xh = bo.xh.p;
    d.part = bo.part.p;
    d.yh = bo.yh.p;
    d.x = bo.x;
    d.y = bo.y;
    d.ldx = bo.ldx;
    d.ldy = bo.ldy;
    d.r = bo.r;
    d.R = R;
    descs.push_back(d);
    const int32_t ki = (int32_t)k;
    for (int64_t b = 0; b < ceil_div(op->n, kGatherRows); ++b) wg.push_back(make_int2(ki, (int32_t)b));
    for (int64_t b = 0; b < ceil_div(op->n, kGatherRows); ++b) wsc.push_back(make_int2(ki, (int32_t)b));
    if (lp->nxh > 0) {
      for (int32_t l = 0; l < lp->npan; ++l) {
        wf.push_back(make_int2(ki, l));
        cf_.push_back((int64_t)lp->f_M_h[l] * lp->f_nkb_h[l]);
      }
      for (int64_t b = 0; b < ceil_div(lp->nxh * R, 256); ++b) wrs.push_back(make_int2(ki, (int32_t)b));
    }
    for (int32_t t = 0; t < bo.ntiles; ++t) {
      wc.push_back(make_int2(ki, t));
      cc_.push_back((int64_t)tiles[t].h * tiles[t].nkb);
    }
    for (int64_t b = 0; b < ceil_div(lp->nyh * R, 256); ++b) wrc.push_back(make_int2(ki, (int32_t)b));
    for (int32_t l = 0; l < op->nleaves; ++l) {
      wb.push_back(make_int2(ki, l));
      cb_.push_back((int64_t)lp->leaf_n_h[l] * lp->b_nkb_h[l]);
    }
    if (lp->ntctiles > 0) {  // the factor pass keeps the upload's tiling (one tile per output slot)
      const int32_t fi = nops + (int32_t)fdescs.size();
      fdescs.push_back(factor_desc(lp, d, lp->tctiles.p, e));
      for (size_t t = 0; t < lp->tchunks.size(); ++t) {
        wfc.push_back(make_int2(fi, (int32_t)t));
        cfc_.push_back((int64_t)lp->tchunks[t].h * lp->tchunks[t].nkb_all);
      }
    }
    if (lp->ntftiles > 0) {
      const int32_t fi = nops + (int32_t)fdescs.size();
      fdescs.push_back(factor_desc(lp, d, lp->tftiles.p, e));
      for (int32_t t = 0; t < lp->ntftiles; ++t) wff.push_back(make_int2(fi, t));
    }
  }
  descs.insert(descs.end(), fdescs.begin(), fdescs.end());
  order_work(wf, cf_, cfg.order);
  order_work(wfc, cfc_, cfg.order);
  order_work(wc, cc_, cfg.order);
  order_work(wb, cb_, cfg.order);
  if ((rc = B->desc.upload(descs, s)) || (rc = B->w_gather.upload(wg, s)) || (rc = B->w_forward.upload(wf, s)) ||
      (rc = B->w_rseg.upload(wrs, s)) || (rc = B->w_ffac.upload(wff, s)) || (rc = B->w_fcoup.upload(wfc, s)) ||
      (rc = B->w_coup.upload(wc, s)) || (rc = B->w_rcoup.upload(wrc, s)) ||
      (rc = B->w_backward.upload(wb, s)) || (rc = B->w_scatter.upload(wsc, s)))
    return rc;
  UHM_HIP(hipStreamSynchronize(s));
  B->cfg = cfg;
  B->configured = true;
  if (B->exec) {
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  if (B->graph) {
    (void)hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
  return UHM_OK;
}

template <int ST, int NT>
void batch_launch_t(LowpBatch* B, hipStream_t s) {
  using V = typename Tr<ST>::V;
  const LpDesc* D = B->desc.p;
  auto go = [&](auto kern, const DevArray<int2>& w, int threads) {
    if (w.n > 0) hipLaunchKernelGGL(kern, dim3((unsigned)w.n), dim3(threads), 0, s, D, w.p);
  };
  go(k_lpb_gather<ST>, B->w_gather, 256);
  go(k_lpb_forward<ST, NT>, B->w_forward, 64 * kLpWaves);
  go(k_lpb_reduce_segments<ST>, B->w_rseg, 256);
  go(k_lpb_factor<ST, NT>, B->w_ffac, 64 * kLpWaves);  // factored couplings, first pass
  go(k_lpb_coupling<ST, NT, typename Tr<ST>::VB>, B->w_fcoup, 64 * kLpWaves);
  go(k_lpb_coupling<ST, NT, V>, B->w_coup, 64 * kLpWaves);
  go(k_lpb_reduce_coupling<ST>, B->w_rcoup, 256);
  go(k_lpb_backward<ST, NT>, B->w_backward, 64 * kLpWaves);
  go(k_lpb_scatter<V>, B->w_scatter, 256);
}

template <int ST>
void batch_launch_st(LowpBatch* B, hipStream_t s) {
  switch (B->R / 16) {
    case 1: batch_launch_t<ST, 1>(B, s); break;
    case 2: batch_launch_t<ST, 2>(B, s); break;
    case 3: batch_launch_t<ST, 3>(B, s); break;
    default: batch_launch_t<ST, 4>(B, s); break;
  }
}

void batch_launch(LowpBatch* B, hipStream_t s) {
  if (B->storage == UHM_C64)
    batch_launch_st<UHM_C64>(B, s);
  else if (B->storage == UHM_BF16PAIR)
    batch_launch_st<UHM_BF16PAIR>(B, s);
  else
    batch_launch_st<UHM_C128_MULTI>(B, s);
}

}  // namespace

void lowp_batch_delete(LowpBatch* b) { delete b; }

// ---------------------------------------------------------------- products of a solver step
namespace {

// Pinned staging of the step products' descriptors and work lists (grow-only, never
// released); ev marks when the last upload from it has been read.
struct StepProducts {
  unsigned char* dev = nullptr;
  unsigned char* host = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
  bool recorded = false;
};
StepProducts& step_products() {
  static StepProducts* sp = new StepProducts;
  return *sp;
}

template <int ST, int NT>
void step_launch(const LpDesc* D, const int2* const* w, const unsigned* cnt, hipStream_t s) {
  using V = typename Tr<ST>::V;
  auto go = [&](auto kern, int st, int threads) {
    if (cnt[st] > 0) hipLaunchKernelGGL(kern, dim3(cnt[st]), dim3(threads), 0, s, D, w[st]);
  };
  go(k_lpb_gather<ST>, 0, 256);
  go(k_lpb_forward<ST, NT>, 1, 64 * kLpWaves);
  go(k_lpb_reduce_segments<ST>, 2, 256);
  go(k_lpb_factor<ST, NT>, 8, 64 * kLpWaves);  // factored couplings, first pass
  go(k_lpb_coupling<ST, NT, typename Tr<ST>::VB>, 7, 64 * kLpWaves);
  go(k_lpb_coupling<ST, NT, V>, 3, 64 * kLpWaves);
  go(k_lpb_reduce_coupling<ST>, 4, 256);
  go(k_lpb_backward<ST, NT>, 5, 64 * kLpWaves);
  go(k_lpb_scatter<V>, 6, 256);
}

template <int ST>
void step_launch_st(int NT, const LpDesc* D, const int2* const* w, const unsigned* cnt, hipStream_t s) {
  switch (NT) {
    case 1: step_launch<ST, 1>(D, w, cnt, s); break;
    case 2: step_launch<ST, 2>(D, w, cnt, s); break;
    case 3: step_launch<ST, 3>(D, w, cnt, s); break;
    default: step_launch<ST, 4>(D, w, cnt, s); break;
  }
}

}  // namespace

int lowp_step_products(uhm_op* const* ops, const cd* const* const* xcol, cd* const* const* ycol, const int32_t* ncols,
                       int32_t nops, hipStream_t s) {
  if (nops < 1 || !ops || !xcol || !ycol || !ncols) return fail(UHM_EINVAL, "null argument");
  const int storage = ops[0]->lp ? ops[0]->lp->storage : -1;
  int maxc = 0;
  for (int32_t k = 0; k < nops; ++k) {
    if (!ops[k]->lp || ops[k]->lp->storage != storage) return fail(UHM_EINVAL, "step products need one many-RHS form");
    if (ncols[k] < 1 || ncols[k] > kLpRmax) return fail(UHM_EINVAL, "1 to 64 columns per operator");
    for (int32_t q = 0; q < k; ++q)
      if (ops[q] == ops[k]) return fail(UHM_EINVAL, "an operator appears twice in one step product");
    maxc = std::max(maxc, (int)ncols[k]);
  }
  const int R = 16 * ((maxc + 15) / 16);
  const int64_t e = storage == UHM_C128_MULTI ? 16 : 8;
  std::vector<LpDesc> descs, fdescs;
  std::vector<int2> w[9];  // stages 7, 8: the first pass of factored couplings (run after stage 2)
  int rc;
  for (int32_t k = 0; k < nops; ++k) {
    uhm_op* op = ops[k];
    LowpOp* lp = op->lp;
    if ((rc = grow(lp, op->n, std::max(R, lp->wsR)))) return rc;
    LpDesc d = desc_of(op);
    d.ctiles = lp->ctiles.p;
    d.grp_t0 = lp->grp_t0.p;
    d.grp_nt = lp->grp_nt.p;
    d.Xc = lp->Xc.p;
    d.Yc = lp->Yc.p;
    d.p = lp->p.p;
    d.xh = lp->xh.p;
    d.part = lp->part.p;
    d.yh = lp->yh.p;
    d.xcol = xcol[k];
    d.ycol = ycol[k];
    d.r = ncols[k];
    d.R = R;
    descs.push_back(d);
    const int32_t ki = k;
    for (int64_t b = 0; b < ceil_div(op->n, kGatherRows); ++b) w[0].push_back(make_int2(ki, (int32_t)b));
    if (lp->nxh > 0) {
      for (int32_t pn = 0; pn < lp->npan; ++pn) w[1].push_back(make_int2(ki, pn));
      for (int64_t b = 0; b < ceil_div(lp->nxh * R, 256); ++b) w[2].push_back(make_int2(ki, (int32_t)b));
    }
    for (int32_t t = 0; t < lp->nctiles; ++t) w[3].push_back(make_int2(ki, t));
    if (lp->nctiles > 0)
      for (int64_t b = 0; b < ceil_div(lp->nyh * R, 256); ++b) w[4].push_back(make_int2(ki, (int32_t)b));
    for (int32_t l = 0; l < op->nleaves; ++l) w[5].push_back(make_int2(ki, l));
    for (int64_t b = 0; b < ceil_div(op->n, kGatherRows); ++b) w[6].push_back(make_int2(ki, (int32_t)b));
    if (lp->ntctiles > 0) {
      const int32_t fi = nops + (int32_t)fdescs.size();
      fdescs.push_back(factor_desc(lp, d, lp->tctiles.p, e));
      for (int32_t t = 0; t < lp->ntctiles; ++t) w[7].push_back(make_int2(fi, t));
    }
    if (lp->ntftiles > 0) {
      const int32_t fi = nops + (int32_t)fdescs.size();
      fdescs.push_back(factor_desc(lp, d, lp->tftiles.p, e));
      for (int32_t t = 0; t < lp->ntftiles; ++t) w[8].push_back(make_int2(fi, t));
    }
  }
  descs.insert(descs.end(), fdescs.begin(), fdescs.end());
  size_t off[10];
  off[0] = (sizeof(LpDesc) * descs.size() + 15) & ~size_t(15);
  for (int st = 0; st < 9; ++st) off[st + 1] = off[st] + ((sizeof(int2) * w[st].size() + 15) & ~size_t(15));
  const size_t tot = off[9];
  StepProducts& sp = step_products();
  if (sp.recorded) UHM_HIP(hipEventSynchronize(sp.ev));
  if (!sp.ev) UHM_HIP(hipEventCreateWithFlags(&sp.ev, hipEventDisableTiming));
  if (tot > sp.cap) {
    if (sp.dev) (void)hipFree(sp.dev);
    if (sp.host) (void)hipHostFree(sp.host);
    sp.dev = sp.host = nullptr;
    const size_t cap = std::max(tot, 2 * sp.cap + (1 << 16));
    sp.cap = 0;
    UHM_HIP(hipMalloc(reinterpret_cast<void**>(&sp.dev), cap));
    UHM_HIP(hipHostMalloc(reinterpret_cast<void**>(&sp.host), cap, hipHostMallocDefault));
    sp.cap = cap;
  }
  std::memcpy(sp.host, descs.data(), sizeof(LpDesc) * descs.size());
  const int2* dw[9];
  unsigned cnt[9];
  for (int st = 0; st < 9; ++st) {
    std::memcpy(sp.host + off[st], w[st].data(), sizeof(int2) * w[st].size());
    dw[st] = reinterpret_cast<const int2*>(sp.dev + off[st]);
    cnt[st] = (unsigned)w[st].size();
  }
  UHM_HIP(hipMemcpyAsync(sp.dev, sp.host, tot, hipMemcpyHostToDevice, s));
  UHM_HIP(hipEventRecord(sp.ev, s));
  sp.recorded = true;
  const LpDesc* D = reinterpret_cast<const LpDesc*>(sp.dev);
  if (storage == UHM_C64)
    step_launch_st<UHM_C64>(R / 16, D, dw, cnt, s);
  else if (storage == UHM_BF16PAIR)
    step_launch_st<UHM_BF16PAIR>(R / 16, D, dw, cnt, s);
  else
    step_launch_st<UHM_C128_MULTI>(R / 16, D, dw, cnt, s);
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail(UHM_EHIP, std::string("kernel launch: ") + hipGetErrorString(he));
  return UHM_OK;
}

int lowp_batch_create(uhm_op* const* ops, int32_t nops, const void* const* X, const int64_t* ldx, void* const* Y,
                      const int64_t* ldy, const int32_t* nrhs, hipStream_t s, LowpBatch** out) {
  if (!ops || nops < 1 || !X || !Y || !ldx || !ldy || !nrhs || !out) return fail(UHM_EINVAL, "null argument");
  *out = nullptr;
  std::unique_ptr<LowpBatch> B(new (std::nothrow) LowpBatch);
  if (!B) return fail(UHM_ENOMEM, "host allocation");
  int rmax = 1;
  for (int32_t k = 0; k < nops; ++k) {
    if (!ops[k] || !ops[k]->lp) return fail(UHM_EINVAL, "batched operators must use a many-RHS storage form");
    if (ops[k]->storage != ops[0]->storage) return fail(UHM_EINVAL, "batched operators must share one storage form");
    if (nrhs[k] < 1 || nrhs[k] > kLpRmax) return fail(UHM_EINVAL, "nrhs must be in [1, 64] per operator");
    if (!X[k] || !Y[k] || ldx[k] < ops[k]->n || ldy[k] < ops[k]->n) return fail(UHM_EINVAL, "bad vector or leading dimension");
    rmax = std::max(rmax, (int)nrhs[k]);
  }
  B->storage = ops[0]->lp->storage;  // the kernels of the base form (factored forms included)
  B->R = 16 * ((rmax + 15) / 16);
  const int64_t e = B->storage == UHM_C128_MULTI ? 16 : 8;
  std::string sig = "st" + std::to_string(B->storage) + "R" + std::to_string(B->R);
  for (int32_t k = 0; k < nops; ++k) {
    std::unique_ptr<BatchOp> bo(new (std::nothrow) BatchOp);
    if (!bo) return fail(UHM_ENOMEM, "host allocation");
    uhm_op* op = ops[k];
    LowpOp* lp = op->lp;
    bo->op = op;
    bo->x = X[k];
    bo->y = Y[k];
    bo->ldx = ldx[k];
    bo->ldy = ldy[k];
    bo->r = nrhs[k];
    const int64_t R = B->R;
    int rc;
    if ((rc = bo->Xc.alloc(e * op->n * R)) || (rc = bo->Yc.alloc(e * op->n * R)) ||
        (rc = bo->p.alloc(e * std::max<int64_t>(1, lp->p_rows * R))) ||
        (rc = bo->xh.alloc(e * std::max<int64_t>(1, (lp->nxh + lp->ntf) * R))) ||
        (rc = bo->yh.alloc(e * std::max<int64_t>(1, lp->nyh * R))))
      return rc;
    sig += "|" + std::to_string(op->n) + "," + std::to_string(lp->nxh) + "," + std::to_string(lp->nyh) + "," +
           std::to_string(lp->chunks.size()) + "," + std::to_string(lp->tchunks.size()) + "," + std::to_string(nrhs[k]);
    B->ops.push_back(std::move(bo));
  }
  B->signature = sig;
  BatchConfig cfg;
  auto it = tune_cache().find(sig);
  if (it != tune_cache().end()) cfg = it->second;
  int rc = configure(B.get(), cfg, s);
  if (rc) return rc;
  *out = B.release();
  return UHM_OK;
}

int lowp_batch_run(LowpBatch* B, hipStream_t s) {
  if (B->exec) {
    UHM_HIP(hipGraphLaunch(B->exec, s));
  } else {
    batch_launch(B, s);
  }
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail(UHM_EHIP, std::string("batched launch: ") + hipGetErrorString(he));
  return UHM_OK;
}

int lowp_batch_capture(LowpBatch* B, hipStream_t s) {
  if (!s) return fail(UHM_EINVAL, "graph capture needs a non-default stream");
  if (B->exec) return UHM_OK;
  UHM_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  batch_launch(B, s);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  if (e != hipSuccess) return fail(UHM_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  B->graph = g;
  UHM_HIP(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
  return UHM_OK;
}

// Time every candidate schedule (width x order) on the device and keep the fastest; the
// winner is cached for batches of the same signature in this process.
int lowp_batch_tune(LowpBatch* B, hipStream_t s, int32_t* width_out, int32_t* order_out, double* ms_out) {
  auto it = tune_cache().find(B->signature);
  BatchConfig best;
  double best_ms = -1.0;
  if (it != tune_cache().end()) {
    best = it->second;
  } else {
    hipEvent_t a, b;
    UHM_HIP(hipEventCreate(&a));
    UHM_HIP(hipEventCreate(&b));
    for (int32_t wdt : kTileWidths)
      for (int32_t ord = 0; ord < 3; ++ord) {
        BatchConfig c;
        c.coup_cols = wdt;
        c.order = ord;
        int rc = configure(B, c, s);
        if (rc) {
          (void)hipEventDestroy(a);
          (void)hipEventDestroy(b);
          return rc;
        }
        batch_launch(B, s);  // warm
        UHM_HIP(hipEventRecord(a, s));
        for (int rep = 0; rep < 3; ++rep) batch_launch(B, s);
        UHM_HIP(hipEventRecord(b, s));
        UHM_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        UHM_HIP(hipEventElapsedTime(&ms, a, b));
        ms /= 3.f;
        if (best_ms < 0.0 || ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    tune_cache()[B->signature] = best;
  }
  int rc = configure(B, best, s);
  if (rc) return rc;
  if (width_out) *width_out = best.coup_cols;
  if (order_out) *order_out = best.order;
  if (ms_out) *ms_out = best_ms;
  return UHM_OK;
}

}  // namespace uhm_detail

using namespace uhm_detail;

extern "C" {

int uhm_batch_create(uhm_op* const* ops, int32_t nops, const void* const* X, const int64_t* ldx, void* const* Y,
                     const int64_t* ldy, const int32_t* nrhs, void* hip_stream, uhm_batch** out) {
  if (!out) return fail(UHM_EINVAL, "null argument");
  LowpBatch* b = nullptr;
  const int rc = lowp_batch_create(ops, nops, X, ldx, Y, ldy, nrhs, static_cast<hipStream_t>(hip_stream), &b);
  *out = reinterpret_cast<uhm_batch*>(b);
  return rc;
}

int uhm_batch_run(uhm_batch* b, void* hip_stream) {
  if (!b) return fail(UHM_EINVAL, "null batch");
  return lowp_batch_run(reinterpret_cast<LowpBatch*>(b), static_cast<hipStream_t>(hip_stream));
}

int uhm_batch_tune(uhm_batch* b, void* hip_stream, int32_t* tile_width, int32_t* order, double* best_ms) {
  if (!b) return fail(UHM_EINVAL, "null batch");
  return lowp_batch_tune(reinterpret_cast<LowpBatch*>(b), static_cast<hipStream_t>(hip_stream), tile_width, order,
                         best_ms);
}

int uhm_batch_capture(uhm_batch* b, void* hip_stream) {
  if (!b) return fail(UHM_EINVAL, "null batch");
  return lowp_batch_capture(reinterpret_cast<LowpBatch*>(b), static_cast<hipStream_t>(hip_stream));
}

void uhm_batch_free(uhm_batch* b) { lowp_batch_delete(reinterpret_cast<LowpBatch*>(b)); }

}  // extern "C"
