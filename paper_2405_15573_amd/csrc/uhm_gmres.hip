// Batched restarted GMRES(m) and mixed-precision GMRES with iterative refinement.
//
// Every right-hand side has its own Krylov space; all of them advance in lockstep so that
// each Arnoldi step is one batched product with the operator (uhm_matvec over nrhs
// columns) plus batched FP64 kernels.  The basis is orthogonalised by classical
// Gram-Schmidt applied twice, with the second pass of each vector delayed by one step and
// fused with the first pass of the next (the one-reduction "DCGS2" scheme of Swirydowicz,
// Langou, Ananthan, Yang and Thomas, and of Bielich et al.): at step j the last vector
// t = V_j has had one projection, and w = A t.  One sweep over the basis forms
// a = V^* t and b = V^* w (basis vectors 0 .. j-1), t^* t and t^* w; one sweep forms
// the final V_j = (t - V a) / r_j, r_j = sqrt(t^* t - |a|^2), and the projected
// w = (I - V V^*) w / r_j over V_0 .. V_j, with its norm.  The basis is read twice per
// step instead of twice per projection.  The Hessenberg column of step j - 1 becomes final
// at step j (the delayed projection changes it), so its Givens rotation and the residual
// estimate it gives lag one step; at the end of a cycle one more sweep finalises the last
// column without a product.  Partial sums are per wavefront over fixed row ranges and are
// reduced in a fixed order (deterministic).
// The (m+1) x m Hessenberg matrices, the Givens rotations and the small triangular solves
// stay on the device in FP64: a step's coefficients never leave the GPU, and the host
// reads back only the number of columns still running.  A single solve reads that count one
// step late, so the host never waits for the step it has just issued; when the count says
// that every column stopped, at most one further step has been issued, on columns that are
// all inactive, and it changes nothing.
//
// With an inner operator (complex64 or bf16 pairs) the solve is iterative refinement: the
// residual r = b - A x is formed with the FP64 operator, an inner GMRES(m) whose products
// use the low-precision operator (vectors converted to complex64 for the product and back)
// reduces it by inner_tol, and x += d.
#include "uhm_internal.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <cmath>
#include <complex>
#include <map>
#include <tuple>

namespace uhm_detail {
namespace {

using cf = float2;
constexpr int kGB = 256;      // threads per block
constexpr int kGRows = 2048;  // rows per block in the batched reductions

// A DPP rotation by N lanes within each 16-lane row.
template <int N>
__device__ __forceinline__ double row_ror(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x120 + N, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x120 + N, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum of v over the 64 lanes of the wave (all lanes active), the same value in every lane.
// Lane moves only, no LDS: the gfx950 lane swaps add the two halves (v_permlane32_swap)
// and then the row pairs (v_permlane16_swap), so each lane holds the sum of its four lanes
// L mod 16 + 16 k; four DPP rotations sum each 16-lane row; lane 0's total is broadcast.
// The order of the additions is fixed.
__device__ __forceinline__ double warp_sum(double v) {
  {
    const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  }
  {
    const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(v), __double2loint(v), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(v), __double2hiint(v), false, false);
    v = __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
  }
  v += row_ror<8>(v);
  v += row_ror<4>(v);
  v += row_ror<2>(v);
  v += row_ror<1>(v);
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}

// Block-wide sum of (re, im) into (out[0], out[1]) of thread 0; fixed order.
__device__ __forceinline__ void block_sum2(double re, double im, double* sh, double& ore, double& oim) {
  re = warp_sum(re);
  im = warp_sum(im);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sh[2 * w] = re;
    sh[2 * w + 1] = im;
  }
  __syncthreads();
  ore = oim = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < kGB / 64; ++q) {
      ore += sh[2 * q];
      oim += sh[2 * q + 1];
    }
}

// ---- Arnoldi kernels: one wavefront per kAWRows rows of one column, kAPer rows per lane
constexpr int kAWRows = 512;
constexpr int kAPer = kAWRows / 64;

// Step j (>= 0) of column c, rows of wave sb: partial sums of a_i = V_i^* t and
// b_i = V_i^* w for i < j, of t^* w and of t^* t, where t = V_j.  Entry e of the column,
// at part[(e r + c) nsub + sb]: a_e (e < j), b_{e-j} (j <= e < 2j), t^* w (2j), t^* t
// (2j + 1, real).  Columns that have stopped are skipped.
__device__ __forceinline__ void a_dots_body(int sb, int c, const cd* __restrict__ V, int64_t vstride, int j,
                                            const cd* __restrict__ w, int64_t n, int r, int nsub,
                                            const int* __restrict__ act, cd* __restrict__ part) {
  const int lane = threadIdx.x & 63;
  if (sb >= nsub || !act[c]) return;
  const int64_t r0 = (int64_t)sb * kAWRows;
  const int64_t lim = n - r0 - lane;  // rows q * 64 < lim are in range
  const cd* tc = V + (int64_t)j * vstride + (int64_t)c * n + r0 + lane;
  const cd* wc = w + (int64_t)c * n + r0 + lane;
  cd tv[kAPer], wv[kAPer];
  double tt = 0.0, twr = 0.0, twi = 0.0;
#pragma unroll
  for (int q = 0; q < kAPer; ++q) {
    const bool ok = q * 64 < lim;
    tv[q] = ok ? tc[q * 64] : make_double2(0.0, 0.0);
    wv[q] = ok ? wc[q * 64] : make_double2(0.0, 0.0);
    tt = fma(tv[q].x, tv[q].x, fma(tv[q].y, tv[q].y, tt));
    twr = fma(tv[q].x, wv[q].x, fma(tv[q].y, wv[q].y, twr));
    twi = fma(tv[q].x, wv[q].y, fma(-tv[q].y, wv[q].x, twi));
  }
  auto put = [&](int e, double re, double im) {
    re = warp_sum(re);
    im = warp_sum(im);
    if (lane == 0) part[((int64_t)e * r + c) * nsub + sb] = make_double2(re, im);
  };
  for (int i = 0; i < j; ++i) {
    const cd* vi = V + (int64_t)i * vstride + (int64_t)c * n + r0 + lane;
    cd v[kAPer];
#pragma unroll
    for (int q = 0; q < kAPer; ++q) v[q] = q * 64 < lim ? vi[q * 64] : make_double2(0.0, 0.0);
    double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
#pragma unroll
    for (int q = 0; q < kAPer; ++q) {
      ar = fma(v[q].x, tv[q].x, fma(v[q].y, tv[q].y, ar));
      ai = fma(v[q].x, tv[q].y, fma(-v[q].y, tv[q].x, ai));
      br = fma(v[q].x, wv[q].x, fma(v[q].y, wv[q].y, br));
      bi = fma(v[q].x, wv[q].y, fma(-v[q].y, wv[q].x, bi));
    }
    put(i, ar, ai);
    put(j + i, br, bi);
  }
  put(2 * j, twr, twi);
  put(2 * j + 1, tt, 0.0);
}

__global__ __launch_bounds__(kGB) void k_a_dots(const cd* __restrict__ V, int64_t vstride, int j,
                                                const cd* __restrict__ w, int64_t n, int r, int nsub,
                                                const int* __restrict__ act, cd* __restrict__ part) {
  a_dots_body(blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), blockIdx.y, V, vstride, j, w, n, r, nsub, act, part);
}

// out[q] = sum_sb part[q nsub + sb], q = e r + c, for the running columns.
__device__ __forceinline__ void a_reduce_body(int64_t q, const cd* __restrict__ part, int nsub, int64_t nq, int r,
                                              const int* __restrict__ act, cd* __restrict__ out) {
  if (q >= nq) return;
  double re = 0.0, im = 0.0;
  if (act[q % r])
    for (int sb = 0; sb < nsub; ++sb) {
      const cd v = part[q * nsub + sb];
      re += v.x;
      im += v.y;
    }
  out[q] = make_double2(re, im);
}
__global__ __launch_bounds__(kGB) void k_a_reduce(const cd* __restrict__ part, int nsub, int64_t nq, int r,
                                                  const int* __restrict__ act, cd* __restrict__ out) {
  a_reduce_body((int64_t)blockIdx.x * kGB + threadIdx.x, part, nsub, nq, r, act, out);
}

// Step j of column c, rows of wave sb, with the column's update coefficients
// (coef[e r + c]: gv_i (e = i < j), gw_i (e = j + i), sv (2j), sw (2j + 1), gt (2j + 2)):
//   V_j = sv t + sum_i gv_i V_i   (j > 0; V_0 is final from the start of the cycle)
//   w   = sw w + gt t + sum_i gw_i V_i
// with t = V_j before the update; partial ||w||^2 at w2[c nsub + sb].  Each wave reads
// and writes its own rows only.
__device__ __forceinline__ void a_update_body(int sb, int c, cd* __restrict__ V, int64_t vstride, int j,
                                              const cd* __restrict__ coef, cd* __restrict__ w, int64_t n, int r,
                                              int nsub, const int* __restrict__ act, double* __restrict__ w2) {
  const int lane = threadIdx.x & 63;
  if (sb >= nsub || !act[c]) return;
  const int64_t r0 = (int64_t)sb * kAWRows;
  const int64_t lim = n - r0 - lane;
  cd* tc = V + (int64_t)j * vstride + (int64_t)c * n + r0 + lane;
  cd* wc = w + (int64_t)c * n + r0 + lane;
  const double sv = coef[(int64_t)(2 * j) * r + c].x, sw = coef[(int64_t)(2 * j + 1) * r + c].x;
  const cd gt = coef[(int64_t)(2 * j + 2) * r + c];
  cd tv[kAPer], wv[kAPer];
#pragma unroll
  for (int q = 0; q < kAPer; ++q) {
    const bool ok = q * 64 < lim;
    const cd t = ok ? tc[q * 64] : make_double2(0.0, 0.0);
    const cd x = ok ? wc[q * 64] : make_double2(0.0, 0.0);
    tv[q] = make_double2(sv * t.x, sv * t.y);
    wv[q] = make_double2(fma(sw, x.x, gt.x * t.x - gt.y * t.y), fma(sw, x.y, gt.x * t.y + gt.y * t.x));
  }
  for (int i = 0; i < j; ++i) {
    const cd* vi = V + (int64_t)i * vstride + (int64_t)c * n + r0 + lane;
    const cd gv = coef[(int64_t)i * r + c], gw = coef[(int64_t)(j + i) * r + c];
    cd v[kAPer];
#pragma unroll
    for (int q = 0; q < kAPer; ++q) v[q] = q * 64 < lim ? vi[q * 64] : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < kAPer; ++q) {
      tv[q].x = fma(gv.x, v[q].x, fma(-gv.y, v[q].y, tv[q].x));
      tv[q].y = fma(gv.x, v[q].y, fma(gv.y, v[q].x, tv[q].y));
      wv[q].x = fma(gw.x, v[q].x, fma(-gw.y, v[q].y, wv[q].x));
      wv[q].y = fma(gw.x, v[q].y, fma(gw.y, v[q].x, wv[q].y));
    }
  }
  double s2 = 0.0;
#pragma unroll
  for (int q = 0; q < kAPer; ++q)
    if (q * 64 < lim) {
      if (j > 0) tc[q * 64] = tv[q];
      wc[q * 64] = wv[q];
      s2 = fma(wv[q].x, wv[q].x, fma(wv[q].y, wv[q].y, s2));
    }
  s2 = warp_sum(s2);
  if (lane == 0) w2[(int64_t)c * nsub + sb] = s2;
}
__global__ __launch_bounds__(kGB) void k_a_update(cd* __restrict__ V, int64_t vstride, int j,
                                                  const cd* __restrict__ coef, cd* __restrict__ w, int64_t n, int r,
                                                  int nsub, const int* __restrict__ act, double* __restrict__ w2) {
  a_update_body(blockIdx.x * (kGB / 64) + (threadIdx.x >> 6), blockIdx.y, V, vstride, j, coef, w, n, r, nsub, act, w2);
}

// ---- the least-squares problem of a cycle, on the device
// State of one solve's current cycle, column c: the Hessenberg columns as the Arnoldi
// relation A V = V Hu has them, Hu[(c m + j)(m+1) + i] (column j is provisional until step
// j + 1), the same columns rotated, H, the rotated right-hand side g[c (m+1) + i], the
// rotations cs[c m + i], sn[c m + i], active[c] (the column still iterates), jc[c] (final
// columns), rtol[c] (residual estimate at which it stops), scale[c].x = 1 / ||w|| of the
// last step.
struct Lsq {
  cd *H, *Hu, *g, *cs, *sn, *scale, *y;
  int *active, *jc;
  const double* rtol;
  unsigned long long* reorth;  // column-steps whose vector got its second projection
  int m, r;
};

__device__ __forceinline__ cd c_mul(cd a, cd b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) b
__device__ __forceinline__ cd c_cmul(cd a, cd b) { return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__device__ __forceinline__ cd c_add(cd a, cd b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cd c_sub(cd a, cd b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cd c_scale(double s, cd a) { return make_double2(s * a.x, s * a.y); }

// Final column k of column c's Hessenberg matrix: copied from Hu, the earlier rotations
// applied, a new rotation that annihilates the subdiagonal entry, g updated; the column
// stops once its residual estimate |g_{k+1}| reaches rtol[c] or the subdiagonal vanishes.
__device__ __forceinline__ void rotate_column(int c, int k, const Lsq& q) {
  const int m = q.m;
  const cd* hu = q.Hu + ((int64_t)c * m + k) * (m + 1);
  cd* col = q.H + ((int64_t)c * m + k) * (m + 1);
  for (int i = 0; i <= k + 1; ++i) col[i] = hu[i];
  const double hs = hypot(hu[k + 1].x, hu[k + 1].y);
  const cd* csc = q.cs + (int64_t)c * m;
  const cd* snc = q.sn + (int64_t)c * m;
  for (int i = 0; i < k; ++i) {
    const cd a = col[i], b = col[i + 1], ci = csc[i], si = snc[i];
    col[i] = c_add(c_cmul(ci, a), c_cmul(si, b));
    col[i + 1] = c_sub(c_mul(ci, b), c_mul(si, a));
  }
  const cd a = col[k], b = col[k + 1];
  const double den = sqrt((a.x * a.x + a.y * a.y) + (b.x * b.x + b.y * b.y));
  cd ck = make_double2(1.0, 0.0), sk = make_double2(0.0, 0.0);
  if (den > 0.0) {
    ck = make_double2(a.x / den, a.y / den);
    sk = make_double2(b.x / den, b.y / den);
  }
  q.cs[(int64_t)c * m + k] = ck;
  q.sn[(int64_t)c * m + k] = sk;
  col[k] = c_add(c_cmul(ck, a), c_cmul(sk, b));
  col[k + 1] = make_double2(0.0, 0.0);
  cd* gc = q.g + (int64_t)c * (m + 1);
  const cd gk = gc[k];
  gc[k] = c_cmul(ck, gk);
  const cd sg = c_mul(sk, gk);
  gc[k + 1] = make_double2(-sg.x, -sg.y);
  q.jc[c] = k + 1;
  if (hypot(gc[k + 1].x, gc[k + 1].y) <= q.rtol[c] || hs <= 1e-300) q.active[c] = 0;
}

// Step j of column c, one wavefront, from the sums of a_dots_body (dv[e r + c]: a, b,
// t^* w, t^* t).
// 1. j > 0: the delayed projection of t = V_j gives r_j = sqrt(t^* t - |a|^2) and the final
//    V_j = (t - V a) / r_j, so t = V a + r_j V_j: the provisional column j - 1 becomes
//    Hu[i, j-1] += Hu[j, j-1] a_i (i < j), Hu[j, j-1] *= r_j, and is rotated (which may stop
//    the column).  With `tail` (the end of a cycle, no product of V_j) that is all.
// 2. The provisional column j.  A V_j = (w - V z) / r_j with z = Hu a (A applied to V a),
//    so Hu[i, j] = (b_i - z_i) / r_j (i < j) and Hu[j, j] = c_j - z_j / r_j with
//    c_j = V_j^* w / r_j = (t^* w - a^* b) / r_j^2.  The projected vector
//    (I - V V^*) A V_j = (I - V V^*) w / r_j = (w - c_j t - sum_i (b_i - c_j a_i) V_i) / r_j
//    gives the update coefficients of a_update_body.
__device__ __forceinline__ void step_body(int c, int j, const cd* __restrict__ dv, cd* __restrict__ coef, bool tail,
                                          const Lsq& q) {
  const int lane = threadIdx.x & 63;
  if (c >= q.r || !q.active[c]) return;
  const int m = q.m, r = q.r;
  auto A = [&](int i) { return dv[(int64_t)i * r + c]; };
  auto B = [&](int i) { return dv[(int64_t)(j + i) * r + c]; };
  double rj = 1.0;
  if (j > 0) {
    double aa = 0.0;
    for (int i = lane; i < j; i += 64) {
      const cd ai = A(i);
      aa = fma(ai.x, ai.x, fma(ai.y, ai.y, aa));
    }
    aa = warp_sum(aa);
    const double rho2 = dv[(int64_t)(2 * j + 1) * r + c].x - aa;
    rj = rho2 > 0.0 ? sqrt(rho2) : 0.0;
    cd* hp = q.Hu + ((int64_t)c * m + (j - 1)) * (m + 1);
    const cd hs = hp[j];
    for (int i = lane; i < j; i += 64) hp[i] = c_add(hp[i], c_mul(hs, A(i)));
    __syncthreads();
    if (lane == 0) {
      hp[j] = c_scale(rj, hs);
      atomicAdd(q.reorth, 1ull);
      rotate_column(c, j - 1, q);
    }
    __syncthreads();
    if (tail || !q.active[c]) return;
  }
  const double ir = 1.0 / rj;
  double abr = 0.0, abi = 0.0;  // a^* b
  for (int i = lane; i < j; i += 64) {
    const cd t = c_cmul(A(i), B(i));
    abr += t.x;
    abi += t.y;
  }
  abr = warp_sum(abr);
  abi = warp_sum(abi);
  const cd tw = dv[(int64_t)(2 * j) * r + c];
  const cd cj = c_scale(ir * ir, make_double2(tw.x - abr, tw.y - abi));
  cd* hj = q.Hu + ((int64_t)c * m + j) * (m + 1);
  for (int k = lane; k <= j; k += 64) {
    // z_k = sum_i Hu[k, i] a_i over the columns i < j with an entry in row k (i >= k - 1)
    cd z = make_double2(0.0, 0.0);
    for (int i = k > 0 ? k - 1 : 0; i < j; ++i) z = c_add(z, c_mul(q.Hu[((int64_t)c * m + i) * (m + 1) + k], A(i)));
    hj[k] = k < j ? c_scale(ir, c_sub(B(k), z)) : c_sub(cj, c_scale(ir, z));
  }
  for (int i = lane; i < j; i += 64) {
    const cd ai = A(i), bi = B(i);
    coef[(int64_t)i * r + c] = c_scale(-ir, ai);
    coef[(int64_t)(j + i) * r + c] = c_scale(-ir, c_sub(bi, c_mul(cj, ai)));
  }
  if (lane == 0) {
    coef[(int64_t)(2 * j) * r + c] = make_double2(ir, 0.0);
    coef[(int64_t)(2 * j + 1) * r + c] = make_double2(ir, 0.0);
    coef[(int64_t)(2 * j + 2) * r + c] = c_scale(-ir, cj);
  }
}
__global__ __launch_bounds__(64) void k_a_step(int j, const cd* __restrict__ dv, cd* __restrict__ coef, int tail,
                                               Lsq q) {
  step_body(blockIdx.x, j, dv, coef, tail != 0, q);
}

// Step j, column c: ||w|| from the partial sums, the provisional subdiagonal entry
// Hu[j + 1, j] and scale[c] = 1 / ||w|| (0 when w vanished, or the column stopped).
__device__ __forceinline__ void norm_body(int c, int j, const double* __restrict__ w2, int nsub, const Lsq& q) {
  if (c >= q.r) return;
  if (!q.active[c]) {
    q.scale[c] = make_double2(0.0, 0.0);
    return;
  }
  double s = 0.0;
  for (int sb = 0; sb < nsub; ++sb) s += w2[(int64_t)c * nsub + sb];
  const double hn = sqrt(s);
  q.Hu[((int64_t)c * q.m + j) * (q.m + 1) + j + 1] = make_double2(hn, 0.0);
  q.scale[c] = make_double2(hn > 1e-300 ? 1.0 / hn : 0.0, 0.0);
}
__global__ void k_a_norm(int j, const double* __restrict__ w2, int nsub, Lsq q) {
  norm_body(blockIdx.x * blockDim.x + threadIdx.x, j, w2, nsub, q);
}

// count[0] = number of running columns (one wavefront)
__global__ __launch_bounds__(64) void k_a_count(const int* __restrict__ active, int r, int* __restrict__ count) {
  int v = 0;
  for (int c = threadIdx.x; c < r; c += 64) v += active[c] != 0;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (threadIdx.x == 0) count[0] = v;
}

// End of a cycle: y_c = R_c^{-1} g_c by back substitution over the jc[c] steps of column c,
// written to y[i r + c] for i < jm (zero beyond jc[c]).
__device__ __forceinline__ void lsq_body(int c, int jm, const Lsq& q) {
  if (c >= q.r) return;
  const int m = q.m, r = q.r, k = q.jc[c];
  const cd* Hc = q.H + (int64_t)c * m * (m + 1);
  const cd* gc = q.g + (int64_t)c * (m + 1);
  for (int i = jm - 1; i >= k; --i) q.y[(int64_t)i * r + c] = make_double2(0.0, 0.0);
  for (int i = k - 1; i >= 0; --i) {
    cd acc = gc[i];
    for (int t = i + 1; t < k; ++t) acc = c_sub(acc, c_mul(Hc[(int64_t)t * (m + 1) + i], q.y[(int64_t)t * r + c]));
    const cd dg = Hc[(int64_t)i * (m + 1) + i];
    const double dd = dg.x * dg.x + dg.y * dg.y;
    q.y[(int64_t)i * r + c] =
        dd > 0.0 ? make_double2((acc.x * dg.x + acc.y * dg.y) / dd, (acc.y * dg.x - acc.x * dg.y) / dd)
                 : make_double2(0.0, 0.0);
  }
}
__global__ void k_a_lsq(int jm, Lsq q) { lsq_body(blockIdx.x * blockDim.x + threadIdx.x, jm, q); }

// Start of a cycle from the residual norms beta: g = beta e_1, no steps, the column runs
// unless beta <= rtol[c]; sc0[c] = 1 / beta (0 when beta = 0) scales the first vector.
__device__ __forceinline__ void cycle_init_body(int c, const double* __restrict__ beta, const Lsq& q,
                                                double* __restrict__ sc0) {
  if (c >= q.r) return;
  const double b = beta[c];
  cd* gc = q.g + (int64_t)c * (q.m + 1);
  gc[0] = make_double2(b, 0.0);
  for (int i = 1; i <= q.m; ++i) gc[i] = make_double2(0.0, 0.0);
  q.jc[c] = 0;
  q.active[c] = !(b <= q.rtol[c]);
  sc0[c] = b > 0.0 ? 1.0 / b : 0.0;
}
__global__ void k_a_cycle_init(const double* __restrict__ beta, Lsq q, double* __restrict__ sc0) {
  cycle_init_body(blockIdx.x * blockDim.x + threadIdx.x, beta, q, sc0);
}

// ---- the same Arnoldi step for many solves in one launch per kernel
// One solve's buffers: the reduced sums dv, the update coefficients coef, the partial norms
// nrm (r nsub), vnext = V_{j+1}.
struct ArnDesc {
  cd *V, *w, *part, *dv, *coef, *vnext;
  double* nrm;
  int* count;  // the solve's running-column count, in the area copied to the host
  Lsq q;
  int64_t n, vstride;
  int32_t r, nsub, j;
};

// work item of the row kernels: (solve, column, block of kGB/64 row ranges)
__global__ __launch_bounds__(kGB) void k_ab_dots(const ArnDesc* __restrict__ D, const int4* __restrict__ work) {
  const int4 wk = work[blockIdx.x];
  const ArnDesc& d = D[wk.x];
  const int sb = wk.z * (kGB / 64) + (threadIdx.x >> 6);
  a_dots_body(sb, wk.y, d.V, d.vstride, d.j, d.w, d.n, d.r, d.nsub, d.q.active, d.part);
}
__global__ __launch_bounds__(kGB) void k_ab_update(const ArnDesc* __restrict__ D, const int4* __restrict__ work) {
  const int4 wk = work[blockIdx.x];
  const ArnDesc& d = D[wk.x];
  const int sb = wk.z * (kGB / 64) + (threadIdx.x >> 6);
  a_update_body(sb, wk.y, d.V, d.vstride, d.j, d.coef, d.w, d.n, d.r, d.nsub, d.q.active, d.nrm);
}
// work item: (solve, block of kGB entries of the sums)
__global__ __launch_bounds__(kGB) void k_ab_reduce(const ArnDesc* __restrict__ D, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const ArnDesc& d = D[wk.x];
  a_reduce_body((int64_t)wk.y * kGB + threadIdx.x, d.part, d.nsub, (int64_t)(2 * d.j + 2) * d.r, d.r, d.q.active,
                d.dv);
}
// work item: (solve, column), one wavefront
__global__ __launch_bounds__(64) void k_ab_step(const ArnDesc* __restrict__ D, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const ArnDesc& d = D[wk.x];
  step_body(wk.y, d.j, d.dv, d.coef, false, d.q);
}
// work item: (solve, block of 64 columns)
__global__ __launch_bounds__(64) void k_ab_norm(const ArnDesc* __restrict__ D, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const ArnDesc& d = D[wk.x];
  norm_body(wk.y * 64 + threadIdx.x, d.j, d.nrm, d.nsub, d.q);
}
// d.vnext[:, c] = d.w[:, c] * d.q.scale[c].x; work item: (solve, block of kGB elements)
__global__ __launch_bounds__(kGB) void k_ab_scale(const ArnDesc* __restrict__ D, const int2* __restrict__ work) {
  const int2 wk = work[blockIdx.x];
  const ArnDesc& d = D[wk.x];
  const int64_t q = (int64_t)wk.y * kGB + threadIdx.x;
  if (q >= d.n * d.r) return;
  const double sc = d.q.scale[q / d.n].x;
  const cd v = d.w[q];
  d.vnext[q] = make_double2(v.x * sc, v.y * sc);
}
// work item: one solve; its running-column count into d.count
__global__ __launch_bounds__(64) void k_ab_count(const ArnDesc* __restrict__ D) {
  const ArnDesc& d = D[blockIdx.x];
  int v = 0;
  for (int c = threadIdx.x; c < d.r; c += 64) v += d.q.active[c] != 0;
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (threadIdx.x == 0) d.count[0] = v;
}

// nrm_out[c] = sqrt(sum_ch nrm[c * nch + ch])
__global__ void k_g_norm(const double* __restrict__ nrm, int nch, int r, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= r) return;
  double s = 0.0;
  for (int ch = 0; ch < nch; ++ch) s += nrm[(int64_t)c * nch + ch];
  out[c] = sqrt(s);
}

// dst[:, c] = src[:, c] * scale[c]  (scale = 0 where the divisor vanished)
__global__ __launch_bounds__(kGB) void k_g_scale(const cd* __restrict__ src, const double* __restrict__ scale, int64_t n,
                                                 int r, cd* __restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q >= n * r) return;
  const double s = scale[q / n];
  const cd v = src[q];
  dst[q] = make_double2(v.x * s, v.y * s);
}

// dst[:, c] = src[:, c] * scale[c].x
__global__ __launch_bounds__(kGB) void k_g_scale2(const cd* __restrict__ src, const cd* __restrict__ scale, int64_t n,
                                                  int r, cd* __restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q >= n * r) return;
  const double sc = scale[q / n].x;
  const cd v = src[q];
  dst[q] = make_double2(v.x * sc, v.y * sc);
}

// x[:, c] += sum_i V_i[:, c] y[i * r + c]
__global__ __launch_bounds__(kGB) void k_g_combine(const cd* __restrict__ V, int64_t vstride, int nvec,
                                                   const cd* __restrict__ y, cd* __restrict__ x, int64_t ldx, int64_t n,
                                                   int r) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q >= n * r) return;
  const int c = (int)(q / n);
  const int64_t row = q - (int64_t)c * n;
  cd a = x[(int64_t)c * ldx + row];
  for (int i = 0; i < nvec; ++i) {
    const cd v = V[(int64_t)i * vstride + q];
    const cd yi = y[(int64_t)i * r + c];
    a.x += v.x * yi.x - v.y * yi.y;
    a.y += v.x * yi.y + v.y * yi.x;
  }
  x[(int64_t)c * ldx + row] = a;
}

// dst = a - b (contiguous n x r, or strided sources)
__global__ __launch_bounds__(kGB) void k_g_sub(const cd* __restrict__ a, int64_t lda, const cd* __restrict__ b, int64_t n,
                                               int r, cd* __restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q >= n * r) return;
  const int c = (int)(q / n);
  const int64_t row = q - (int64_t)c * n;
  const cd u = a[(int64_t)c * lda + row], v = b[q];
  dst[q] = make_double2(u.x - v.x, u.y - v.y);
}

__global__ __launch_bounds__(kGB) void k_g_copy_strided(const cd* __restrict__ a, int64_t lda, int64_t n, int r,
                                                        cd* __restrict__ dst) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q >= n * r) return;
  const int c = (int)(q / n);
  dst[q] = a[(int64_t)c * lda + (q - (int64_t)c * n)];
}

__global__ __launch_bounds__(kGB) void k_g_to32(const cd* __restrict__ a, int64_t nq, cf* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q < nq) out[q] = make_float2((float)a[q].x, (float)a[q].y);
}

__global__ __launch_bounds__(kGB) void k_g_to64(const cf* __restrict__ a, int64_t nq, cd* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q < nq) out[q] = make_double2((double)a[q].x, (double)a[q].y);
}

__global__ __launch_bounds__(kGB) void k_g_sqnorm(const cd* __restrict__ a, int64_t n, int nch, double* __restrict__ nrm) {
  __shared__ double sh[2 * kGB / 64];
  const int ch = blockIdx.x, c = blockIdx.y;
  const int64_t r0 = (int64_t)ch * kGRows;
  const int64_t r1 = min(n, r0 + kGRows);
  double acc = 0.0;
  for (int64_t row = r0 + threadIdx.x; row < r1; row += kGB) {
    const cd v = a[(int64_t)c * n + row];
    acc += v.x * v.x + v.y * v.y;
  }
  double sum, dummy;
  block_sum2(acc, 0.0, sh, sum, dummy);
  if (threadIdx.x == 0) nrm[(int64_t)c * nch + ch] = sum;
}

// x[:, c] (ldx) += d[:, c] (contiguous), or = d when `assign`
__global__ __launch_bounds__(kGB) void k_g_add(const cd* __restrict__ d, int64_t n, int r, cd* __restrict__ x, int64_t ldx,
                                               int assign) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q >= n * r) return;
  const int c = (int)(q / n);
  cd* px = x + (int64_t)c * ldx + (q - (int64_t)c * n);
  const cd v = d[q];
  if (assign) {
    *px = v;
  } else {
    px->x += v.x;
    px->y += v.y;
  }
}

unsigned nblk(int64_t q) { return (unsigned)((q + kGB - 1) / kGB); }

using C = std::complex<double>;
using Clock = std::chrono::steady_clock;

// Pinned host memory for the small host <-> device copies of the control values.
template <class T>
struct Pinned {
  T* p = nullptr;
  int alloc(int64_t count) {
    UHM_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), sizeof(T) * (size_t)count, hipHostMallocDefault));
    return UHM_OK;
  }
  ~Pinned() {
    if (p) (void)hipHostFree(p);
  }
};

struct Work {
  int64_t n = 0;
  int r = 0, m = 0, nch = 0, nsub = 0;
  // dv: the reduced sums of a step, coef: its update coefficients (both (2m + 4) r)
  DevArray<cd> V, w, t, d, part, dv, coef, ybuf;
  DevArray<double> nrm, nrm_out, rtol, sc0;
  DevArray<cf> x32, y32;
  // least-squares state of the current cycle (Lsq), on the device
  DevArray<cd> H, Hu, g, cs, sn, scale;
  DevArray<int> active, jc, count;
  DevArray<unsigned long long> reorth;
  Pinned<int> hcount;      // running-column counts of the last two steps (a single solve)
  Pinned<double> hrtol;    // staging of rtol uploads
  Pinned<unsigned long long> hreorth;
  hipEvent_t ev[2] = {nullptr, nullptr};  // the copies of hcount[0], hcount[1] are done
  ~Work() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  Lsq lsq() {
    return Lsq{H.p, Hu.p, g.p, cs.p, sn.p, scale.p, ybuf.p, active.p, jc.p, rtol.p, reorth.p, m, r};
  }
};

int alloc_work(Work& W, int64_t n, int r, int m, bool lowp, hipStream_t s) {
  W.n = n;
  W.r = r;
  W.m = m;
  W.nch = (int)((n + kGRows - 1) / kGRows);
  W.nsub = (int)((n + kAWRows - 1) / kAWRows);
  // a step's sums: 2 j + 2 entries per column, j <= m (the end-of-cycle sweep has j = m);
  // its coefficients: 2 j + 3
  const int64_t nsum = (int64_t)(2 * m + 4) * r;
  int rc;
  if ((rc = W.V.alloc((int64_t)(m + 1) * n * r)) || (rc = W.w.alloc(n * r)) || (rc = W.t.alloc(n * r)) ||
      (rc = W.d.alloc(n * r)) || (rc = W.part.alloc(nsum * W.nsub)) || (rc = W.dv.alloc(nsum)) ||
      (rc = W.coef.alloc(nsum)) || (rc = W.ybuf.alloc((int64_t)(m + 1) * r)) ||
      (rc = W.nrm.alloc((int64_t)r * std::max(W.nch, W.nsub))) || (rc = W.nrm_out.alloc(r)) ||
      (rc = W.rtol.alloc(r)) || (rc = W.sc0.alloc(r)) || (rc = W.H.alloc((int64_t)r * m * (m + 1))) ||
      (rc = W.Hu.alloc((int64_t)r * m * (m + 1))) || (rc = W.g.alloc((int64_t)r * (m + 1))) ||
      (rc = W.cs.alloc((int64_t)r * m)) || (rc = W.sn.alloc((int64_t)r * m)) || (rc = W.scale.alloc(r)) ||
      (rc = W.active.alloc(r)) || (rc = W.jc.alloc(r)) || (rc = W.count.alloc(1)) || (rc = W.reorth.alloc(1)) ||
      (rc = W.hcount.alloc(2)) || (rc = W.hrtol.alloc(r)) || (rc = W.hreorth.alloc(1)))
    return rc;
  if (lowp && ((rc = W.x32.alloc(n * r)) || (rc = W.y32.alloc(n * r)))) return rc;
  for (hipEvent_t& e : W.ev) UHM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  UHM_HIP(hipMemsetAsync(W.reorth.p, 0, sizeof(unsigned long long), s));
  UHM_HIP(hipMemsetAsync(W.active.p, 0, sizeof(int) * (size_t)r, s));
  return UHM_OK;
}

// The per-column stopping thresholds of the current inner solve (host values) to the device.
int upload_rtol(Work& W, const std::vector<double>& rtol, hipStream_t s) {
  // the previous upload from the staging area is complete: every caller has synchronised
  // the stream since (the residual norms it needs)
  std::memcpy(W.hrtol.p, rtol.data(), sizeof(double) * (size_t)W.r);
  UHM_HIP(hipMemcpyAsync(W.rtol.p, W.hrtol.p, sizeof(double) * (size_t)W.r, hipMemcpyHostToDevice, s));
  return UHM_OK;
}

// Column norms of a contiguous n x r array.
int norms(Work& W, const cd* a, std::vector<double>& out, hipStream_t s) {
  hipLaunchKernelGGL(k_g_sqnorm, dim3(W.nch, W.r), dim3(kGB), 0, s, a, W.n, W.nch, W.nrm.p);
  hipLaunchKernelGGL(k_g_norm, dim3((W.r + 63) / 64), dim3(64), 0, s, W.nrm.p, W.nch, W.r, W.nrm_out.p);
  out.resize(W.r);
  UHM_HIP(hipMemcpyAsync(out.data(), W.nrm_out.p, sizeof(double) * W.r, hipMemcpyDeviceToHost, s));
  UHM_HIP(hipStreamSynchronize(s));
  return UHM_OK;
}

}  // namespace
}  // namespace uhm_detail

// ------------------------------------------------------------------ resumable solve
// The solve is a state machine that stops whenever it needs a product.  The caller reads
// the request (vector, output buffer, precision), computes the product any way it likes
// (alone, or batched with the requests of other solves) and calls advance.

struct uhm_krylov {
  using cd = uhm_detail::cd;
  template <class T>
  using DevArray = uhm_detail::DevArray<T>;
  uhm_detail::Work W;
  int64_t n = 0;
  int r = 0;
  double tol = 0.0;
  uhm_gmres_opts o{};
  bool mixed = false;
  hipStream_t s = nullptr;
  DevArray<cd> Bc, xacc, res, rhs;
  // request
  int req = UHM_KRYLOV_DONE;  // UHM_KRYLOV_PRODUCT_HIGH / _LOW / DONE
  const void* req_in = nullptr;
  void* req_out = nullptr;
  // bookkeeping (the least-squares state of a cycle is on the device, in W)
  enum Phase { ITER, CYCLE_END, INNER_FINAL_X, OUTER, FINISHED } phase = FINISHED;
  std::vector<double> bn, rn, rtol, beta;
  std::vector<char> done;
  int j = 0;
  int iters = 0, restarts = 0, refinements = 0, cycles = 0;
  double t_arn = 0.0;
  int status = UHM_OK;
};

namespace uhm_detail {
namespace {

// With inner_cycles > 0, an inner solve of the refinement ends after that many cycles.
bool inner_cycles_spent(const uhm_krylov* K) {
  return K->mixed && K->o.inner_cycles > 0 && K->cycles >= K->o.inner_cycles;
}

// The inner solve is over: x += d, then the true residual from the FP64 product of x.
void inner_finish(uhm_krylov* K) {
  Work& W = K->W;
  hipLaunchKernelGGL(k_g_add, dim3(nblk(K->n * K->r)), dim3(kGB), 0, K->s, W.d.p, K->n, K->r, K->xacc.p, K->n, 0);
  K->phase = uhm_krylov::OUTER;
  K->req = UHM_KRYLOV_PRODUCT_HIGH;
  K->req_in = K->xacc.p;
  K->req_out = W.w.p;
}

// t = current inner residual; start a cycle, or finish the inner solve.
int cycle_start(uhm_krylov* K) {
  Work& W = K->W;
  const int r = K->r, m = K->o.restart;
  const int64_t n = K->n;
  hipStream_t s = K->s;
  int rc;
  if ((rc = norms(W, W.t.p, K->beta, s))) return rc;
  bool all = true;
  for (int c = 0; c < r; ++c) {
    K->done[c] = K->beta[c] <= K->rtol[c];
    all = all && K->done[c];
  }
  if (all || K->iters >= K->o.max_iterations || inner_cycles_spent(K)) {
    // inner solve finished: d is in W.d
    if (K->mixed) {
      inner_finish(K);
    } else {
      K->phase = uhm_krylov::INNER_FINAL_X;
      K->req = UHM_KRYLOV_PRODUCT_HIGH;
      K->req_in = W.d.p;
      K->req_out = W.w.p;
    }
    return UHM_OK;
  }
  if (K->cycles++ > 0) ++K->restarts;
  // g = beta e_1 and V_0 = t / beta per column; the columns with beta <= rtol do not run
  // (the device takes the same decision from the same norms)
  hipLaunchKernelGGL(k_a_cycle_init, dim3((r + 63) / 64), dim3(64), 0, s, W.nrm_out.p, W.lsq(), W.sc0.p);
  hipLaunchKernelGGL(k_g_scale, dim3(nblk(n * r)), dim3(kGB), 0, s, W.t.p, W.sc0.p, n, r, W.V.p);
  (void)m;
  K->j = 0;
  K->phase = uhm_krylov::ITER;
  K->req = K->mixed ? UHM_KRYLOV_PRODUCT_LOW : UHM_KRYLOV_PRODUCT_HIGH;
  K->req_in = W.V.p;
  K->req_out = W.w.p;
  return UHM_OK;
}

// Start an inner solve of A d = rhs_src (contiguous) to the per-column tolerances in K->rtol.
int inner_start(uhm_krylov* K, const cd* rhs_src) {
  Work& W = K->W;
  const int64_t nr = K->n * K->r;
  int rc = upload_rtol(W, K->rtol, K->s);
  if (rc) return rc;
  UHM_HIP(hipMemcpyAsync(K->rhs.p, rhs_src, sizeof(cd) * (size_t)nr, hipMemcpyDeviceToDevice, K->s));
  UHM_HIP(hipMemsetAsync(W.d.p, 0, sizeof(cd) * (size_t)nr, K->s));
  UHM_HIP(hipMemcpyAsync(W.t.p, K->rhs.p, sizeof(cd) * (size_t)nr, hipMemcpyDeviceToDevice, K->s));
  K->cycles = 0;
  return cycle_start(K);
}

// The sums of step j over the running columns: a = V^* t, b = V^* w (basis vectors
// 0 .. j-1), t^* w and t^* t, t = V_j, reduced into W.dv.
void step_sums(uhm_krylov* K, int j, const cd* w) {
  Work& W = K->W;
  const int r = K->r;
  const int64_t n = K->n, vstride = n * r;
  const dim3 gw((unsigned)((W.nsub + kGB / 64 - 1) / (kGB / 64)), (unsigned)r);
  const int64_t nq = (int64_t)(2 * j + 2) * r;
  hipLaunchKernelGGL(k_a_dots, gw, dim3(kGB), 0, K->s, W.V.p, vstride, j, w, n, r, W.nsub, W.active.p, W.part.p);
  hipLaunchKernelGGL(k_a_reduce, dim3(nblk(nq)), dim3(kGB), 0, K->s, W.part.p, W.nsub, nq, r, W.active.p, W.dv.p);
}

// One Arnoldi step after the product W.w = A V_j, all on the solve's stream: the sums, the
// delayed projection of V_j with the final Hessenberg column j - 1 and its rotation, the
// projection of w and the provisional column j, V_{j+1} = w / ||w||, and a copy of the
// running-column count to pinned host memory (slot j % 2, event ev).
int arnoldi_issue(uhm_krylov* K) {
  Work& W = K->W;
  const int r = K->r, j = K->j;
  const int64_t n = K->n, vstride = n * r;
  hipStream_t s = K->s;
  const dim3 gw((unsigned)((W.nsub + kGB / 64 - 1) / (kGB / 64)), (unsigned)r);
  step_sums(K, j, W.w.p);
  hipLaunchKernelGGL(k_a_step, dim3((unsigned)r), dim3(64), 0, s, j, W.dv.p, W.coef.p, 0, W.lsq());
  hipLaunchKernelGGL(k_a_update, gw, dim3(kGB), 0, s, W.V.p, vstride, j, W.coef.p, W.w.p, n, r, W.nsub, W.active.p,
                     W.nrm.p);
  hipLaunchKernelGGL(k_a_norm, dim3((unsigned)((r + 63) / 64)), dim3(64), 0, s, j, W.nrm.p, W.nsub, W.lsq());
  hipLaunchKernelGGL(k_g_scale2, dim3(nblk(n * r)), dim3(kGB), 0, s, W.w.p, W.scale.p, n, r,
                     W.V.p + (int64_t)(j + 1) * vstride);
  hipLaunchKernelGGL(k_a_count, dim3(1), dim3(64), 0, s, W.active.p, r, W.count.p);
  UHM_HIP(hipMemcpyAsync(W.hcount.p + (j & 1), W.count.p, sizeof(int), hipMemcpyDeviceToHost, s));
  UHM_HIP(hipEventRecord(W.ev[j & 1], s));
  return UHM_OK;
}

// After step j has been issued: the next request, or the end of the cycle.  all_done: no
// column runs any more.
int arnoldi_next(uhm_krylov* K, bool all_done) {
  Work& W = K->W;
  const int r = K->r, j = K->j;
  const int64_t n = K->n, vstride = n * r;
  hipStream_t s = K->s;
  K->j = j + 1;
  if (!all_done && K->j < K->o.restart && K->iters < K->o.max_iterations) {
    K->req = K->mixed ? UHM_KRYLOV_PRODUCT_LOW : UHM_KRYLOV_PRODUCT_HIGH;
    K->req_in = W.V.p + (int64_t)K->j * vstride;
    K->req_out = W.w.p;
    return UHM_OK;
  }
  // end of the cycle: the last column is still provisional; the delayed projection of
  // V_jm (no product) makes it final.  Then y_c = R_c^{-1} g_c on the device, d += V y,
  // and the residual t = rhs - A d.
  const int jm = K->j;
  step_sums(K, jm, W.V.p + (int64_t)jm * vstride);
  hipLaunchKernelGGL(k_a_step, dim3((unsigned)r), dim3(64), 0, s, jm, W.dv.p, W.coef.p, 1, W.lsq());
  hipLaunchKernelGGL(k_a_lsq, dim3((r + 63) / 64), dim3(64), 0, s, jm, W.lsq());
  hipLaunchKernelGGL(k_g_combine, dim3(nblk(n * r)), dim3(kGB), 0, s, W.V.p, vstride, jm, W.ybuf.p, W.d.p, n, n, r);
  if (inner_cycles_spent(K)) {
    // the refinement step follows at once: its FP64 residual replaces the inner one
    inner_finish(K);
    return UHM_OK;
  }
  K->phase = uhm_krylov::CYCLE_END;
  K->req = K->mixed ? UHM_KRYLOV_PRODUCT_LOW : UHM_KRYLOV_PRODUCT_HIGH;
  K->req_in = W.d.p;
  K->req_out = W.w.p;
  return UHM_OK;
}

// Process-wide scratch of the batched Arnoldi launches: device descriptors and work lists,
// staged through pinned host memory (grow-only, never released; one step at a time).
struct StepScratch {
  std::mutex mu;
  unsigned char* dev = nullptr;
  unsigned char* host = nullptr;
  size_t cap = 0;
  // column pointers of the step's products; pev marks when their upload has been read
  const cd** pdev = nullptr;
  const cd** phost = nullptr;
  size_t pcap = 0;
  hipEvent_t pev = nullptr;
  bool pev_recorded = false;
};
StepScratch& step_scratch() {
  static StepScratch* ss = new StepScratch;
  return *ss;
}

size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// Offsets of one batched step in the scratch buffers (bytes).
struct ManyLayout {
  size_t o_d, o_row, o_red, o_step, o_col, o_sw, o_g, tot;
  unsigned nrow, nred, nstep, ncol, nsw;
};

// arnoldi_issue for many solves: each kernel is launched once over the work of all of them
// on stream s, the Givens updates and the next basis vectors included; the solves'
// running-column counts are gathered into one area and copied to pinned host memory in one
// transfer.  The caller holds the scratch lock until the step is done.
int arnoldi_issue_many(const std::vector<uhm_krylov*>& iter, hipStream_t s, StepScratch& ss, ManyLayout& Lo) {
  std::vector<ArnDesc> D;
  std::vector<int4> wrow;
  std::vector<int2> wred, wstep, wcol, wsc;
  // layout first: descriptors point into the gather area for their counts
  size_t nrow = 0, nred = 0, nstep = 0, ncol = 0, nsc = 0;
  for (uhm_krylov* K : iter) {
    const int r = K->r;
    nrow += (size_t)r * ((K->W.nsub + kGB / 64 - 1) / (kGB / 64));
    nred += (size_t)(((int64_t)(2 * K->j + 2) * r + kGB - 1) / kGB);
    nstep += (size_t)r;
    ncol += (size_t)((r + 63) / 64);
    nsc += (size_t)((K->n * r + kGB - 1) / kGB);
  }
  Lo.o_d = 0;
  Lo.o_row = align16(sizeof(ArnDesc) * iter.size());
  Lo.o_red = Lo.o_row + align16(sizeof(int4) * nrow);
  Lo.o_step = Lo.o_red + align16(sizeof(int2) * nred);
  Lo.o_col = Lo.o_step + align16(sizeof(int2) * nstep);
  Lo.o_sw = Lo.o_col + align16(sizeof(int2) * ncol);
  Lo.o_g = Lo.o_sw + align16(sizeof(int2) * nsc);  // running-column counts, device -> host
  Lo.tot = Lo.o_g + align16(sizeof(int) * iter.size());
  if (Lo.tot > ss.cap) {
    if (ss.dev) (void)hipFree(ss.dev);
    if (ss.host) (void)hipHostFree(ss.host);
    ss.dev = ss.host = nullptr;
    const size_t cap = std::max(Lo.tot, 2 * ss.cap + (1 << 16));
    ss.cap = 0;
    UHM_HIP(hipMalloc(reinterpret_cast<void**>(&ss.dev), cap));
    UHM_HIP(hipHostMalloc(reinterpret_cast<void**>(&ss.host), cap, hipHostMallocDefault));
    ss.cap = cap;
  }
  int* dcount = reinterpret_cast<int*>(ss.dev + Lo.o_g);
  for (size_t k = 0; k < iter.size(); ++k) {
    uhm_krylov* K = iter[k];
    Work& W = K->W;
    const int r = K->r, j = K->j;
    ArnDesc d{};
    d.V = W.V.p;
    d.w = W.w.p;
    d.part = W.part.p;
    d.dv = W.dv.p;
    d.coef = W.coef.p;
    d.vnext = W.V.p + (int64_t)(j + 1) * K->n * r;
    d.nrm = W.nrm.p;
    d.count = dcount + k;
    d.q = W.lsq();
    d.n = K->n;
    d.vstride = K->n * r;
    d.r = r;
    d.nsub = W.nsub;
    d.j = j;
    D.push_back(d);
    const int ki = (int)k;
    for (int c = 0; c < r; ++c)
      for (int zb = 0; zb < (W.nsub + kGB / 64 - 1) / (kGB / 64); ++zb) wrow.push_back(make_int4(ki, c, zb, 0));
    for (int64_t qb = 0; qb < ((int64_t)(2 * j + 2) * r + kGB - 1) / kGB; ++qb) wred.push_back(make_int2(ki, (int)qb));
    for (int c = 0; c < r; ++c) wstep.push_back(make_int2(ki, c));
    for (int cb = 0; cb < (r + 63) / 64; ++cb) wcol.push_back(make_int2(ki, cb));
    for (int64_t sb = 0; sb < (K->n * r + kGB - 1) / kGB; ++sb) wsc.push_back(make_int2(ki, (int)sb));
  }
  Lo.nrow = (unsigned)wrow.size();
  Lo.nred = (unsigned)wred.size();
  Lo.nstep = (unsigned)wstep.size();
  Lo.ncol = (unsigned)wcol.size();
  Lo.nsw = (unsigned)wsc.size();
  std::memcpy(ss.host + Lo.o_d, D.data(), sizeof(ArnDesc) * D.size());
  std::memcpy(ss.host + Lo.o_row, wrow.data(), sizeof(int4) * wrow.size());
  std::memcpy(ss.host + Lo.o_red, wred.data(), sizeof(int2) * wred.size());
  std::memcpy(ss.host + Lo.o_step, wstep.data(), sizeof(int2) * wstep.size());
  std::memcpy(ss.host + Lo.o_col, wcol.data(), sizeof(int2) * wcol.size());
  std::memcpy(ss.host + Lo.o_sw, wsc.data(), sizeof(int2) * wsc.size());
  UHM_HIP(hipMemcpyAsync(ss.dev, ss.host, Lo.o_g, hipMemcpyHostToDevice, s));
  const ArnDesc* dD = reinterpret_cast<const ArnDesc*>(ss.dev + Lo.o_d);
  const int4* dRow = reinterpret_cast<const int4*>(ss.dev + Lo.o_row);
  const int2* dRed = reinterpret_cast<const int2*>(ss.dev + Lo.o_red);
  const int2* dStep = reinterpret_cast<const int2*>(ss.dev + Lo.o_step);
  const int2* dCol = reinterpret_cast<const int2*>(ss.dev + Lo.o_col);
  hipLaunchKernelGGL(k_ab_dots, dim3(Lo.nrow), dim3(kGB), 0, s, dD, dRow);
  hipLaunchKernelGGL(k_ab_reduce, dim3(Lo.nred), dim3(kGB), 0, s, dD, dRed);
  hipLaunchKernelGGL(k_ab_step, dim3(Lo.nstep), dim3(64), 0, s, dD, dStep);
  hipLaunchKernelGGL(k_ab_update, dim3(Lo.nrow), dim3(kGB), 0, s, dD, dRow);
  hipLaunchKernelGGL(k_ab_norm, dim3(Lo.ncol), dim3(64), 0, s, dD, dCol);
  hipLaunchKernelGGL(k_ab_scale, dim3(Lo.nsw), dim3(kGB), 0, s, dD, reinterpret_cast<const int2*>(ss.dev + Lo.o_sw));
  hipLaunchKernelGGL(k_ab_count, dim3((unsigned)iter.size()), dim3(64), 0, s, dD);
  UHM_HIP(hipMemcpyAsync(ss.host + Lo.o_g, ss.dev + Lo.o_g, sizeof(int) * iter.size(), hipMemcpyDeviceToHost, s));
  return UHM_OK;
}

// After the step's counts have arrived: each solve's next request, or the end of its cycle.
int arnoldi_finish_many(const std::vector<uhm_krylov*>& iter, StepScratch& ss, const ManyLayout& Lo) {
  const int* cnt = reinterpret_cast<const int*>(ss.host + Lo.o_g);
  for (size_t k = 0; k < iter.size(); ++k) {
    uhm_krylov* K = iter[k];
    ++K->iters;
    // the single-solve path reads the previous step's count from this slot
    K->W.hcount.p[K->j & 1] = cnt[k];
    int rc = arnoldi_next(K, cnt[k] == 0);
    if (rc) return iter[k]->status = rc;
  }
  return UHM_OK;
}

// One Arnoldi step of a single solve.  The host checks the running-column count of the
// previous step (its copy finished long before, normally), not of this one: when it is zero,
// this step ran on stopped columns only (its effect is nil) and the cycle ends.
int arnoldi_step(uhm_krylov* K) {
  int rc = arnoldi_issue(K);
  if (rc) return rc;
  ++K->iters;
  bool all_done = false;
  if (K->j > 0) {
    const int slot = (K->j - 1) & 1;
    UHM_HIP(hipEventSynchronize(K->W.ev[slot]));
    if (K->W.hcount.p[slot] == 0) {
      all_done = true;
      --K->iters;
    }
  }
  return arnoldi_next(K, all_done);
}

int advance(uhm_krylov* K) {
  Work& W = K->W;
  const int r = K->r;
  const int64_t n = K->n;
  hipStream_t s = K->s;
  switch (K->phase) {
    case uhm_krylov::ITER:
      return arnoldi_step(K);
    case uhm_krylov::CYCLE_END:
      hipLaunchKernelGGL(k_g_sub, dim3(nblk(n * r)), dim3(kGB), 0, s, K->rhs.p, n, W.w.p, n, r, W.t.p);
      return cycle_start(K);
    case uhm_krylov::INNER_FINAL_X: {
      // plain GMRES: x = d, true residual from the product
      UHM_HIP(hipMemcpyAsync(K->xacc.p, W.d.p, sizeof(cd) * (size_t)(n * r), hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(k_g_sub, dim3(nblk(n * r)), dim3(kGB), 0, s, K->Bc.p, n, W.w.p, n, r, K->res.p);
      int rc = norms(W, K->res.p, K->rn, s);
      if (rc) return rc;
      K->phase = uhm_krylov::FINISHED;
      K->req = UHM_KRYLOV_DONE;
      return UHM_OK;
    }
    case uhm_krylov::OUTER: {
      hipLaunchKernelGGL(k_g_sub, dim3(nblk(n * r)), dim3(kGB), 0, s, K->Bc.p, n, W.w.p, n, r, K->res.p);
      int rc = norms(W, K->res.p, K->rn, s);
      if (rc) return rc;
      ++K->refinements;
      bool all = true;
      for (int c = 0; c < r; ++c) all = all && K->rn[c] <= K->tol * K->bn[c];
      if (all || K->refinements >= K->o.max_refinements || K->iters >= K->o.max_iterations) {
        K->phase = uhm_krylov::FINISHED;
        K->req = UHM_KRYLOV_DONE;
        return UHM_OK;
      }
      for (int c = 0; c < r; ++c) K->rtol[c] = K->o.inner_tol * K->rn[c];
      return inner_start(K, K->res.p);
    }
    default:
      return fail(UHM_EINVAL, "the solve needs no product");
  }
}

}  // namespace
}  // namespace uhm_detail

using namespace uhm_detail;

extern "C" {

int uhm_krylov_create(int64_t n, int32_t nrhs, const void* B, int64_t ldb, double tol, int32_t mixed,
                      const uhm_gmres_opts* opts, void* hip_stream, uhm_krylov** out) {
  if (!out || !B) return fail(UHM_EINVAL, "null argument");
  *out = nullptr;
  if (n < 1 || nrhs < 1 || ldb < n || !(tol > 0.0)) return fail(UHM_EINVAL, "bad n, nrhs, leading dimension or tol");
  uhm_gmres_opts o{50, 2000, 30, 1e-4, 0};
  if (opts) o = *opts;
  if (o.restart < 1 || o.max_iterations < 1 || o.max_refinements < 1 || !(o.inner_tol > 0.0) || o.inner_tol >= 1.0 ||
      o.inner_cycles < 0)
    return fail(UHM_EINVAL, "bad GMRES options");
  std::unique_ptr<uhm_krylov> K(new (std::nothrow) uhm_krylov);
  if (!K) return fail(UHM_ENOMEM, "host allocation");
  K->n = n;
  K->r = nrhs;
  K->tol = tol;
  K->o = o;
  K->mixed = mixed != 0;
  K->s = static_cast<hipStream_t>(hip_stream);
  hipStream_t s = K->s;
  const int r = nrhs, m = o.restart;
  int rc;
  if ((rc = alloc_work(K->W, n, r, m, false, s)) || (rc = K->Bc.alloc(n * r)) || (rc = K->xacc.alloc(n * r)) ||
      (rc = K->res.alloc(n * r)) || (rc = K->rhs.alloc(n * r)))
    return rc;
  K->done.assign(r, 0);
  K->rtol.assign(r, 0.0);
  hipLaunchKernelGGL(k_g_copy_strided, dim3(nblk(n * r)), dim3(kGB), 0, s, static_cast<const cd*>(B), ldb, n, r, K->Bc.p);
  UHM_HIP(hipMemsetAsync(K->xacc.p, 0, sizeof(cd) * (size_t)(n * r), s));
  if ((rc = norms(K->W, K->Bc.p, K->bn, s))) return rc;
  K->rn = K->bn;
  if (K->mixed) {
    bool all = true;
    for (int c = 0; c < r; ++c) all = all && K->bn[c] <= tol * K->bn[c];
    if (all) {
      K->phase = uhm_krylov::FINISHED;
      K->req = UHM_KRYLOV_DONE;
    } else {
      for (int c = 0; c < r; ++c) K->rtol[c] = o.inner_tol * K->bn[c];
      if ((rc = inner_start(K.get(), K->Bc.p))) return rc;
    }
  } else {
    for (int c = 0; c < r; ++c) K->rtol[c] = tol * K->bn[c];
    if ((rc = inner_start(K.get(), K->Bc.p))) return rc;
  }
  *out = K.release();
  return UHM_OK;
}

int uhm_krylov_next(uhm_krylov* K, const void** in, void** out) {
  if (!K) return fail(UHM_EINVAL, "null solve");
  if (in) *in = K->req_in;
  if (out) *out = K->req_out;
  return K->req;
}

int uhm_krylov_advance(uhm_krylov* K) {
  if (!K) return fail(UHM_EINVAL, "null solve");
  const auto t0 = Clock::now();
  const int rc = advance(K);
  K->t_arn += std::chrono::duration<double>(Clock::now() - t0).count();
  if (rc) K->status = rc;
  return rc;
}

int uhm_krylov_result(uhm_krylov* K, void* X, int64_t ldx, uhm_gmres_info* info) {
  if (!K) return fail(UHM_EINVAL, "null solve");
  if (K->phase != uhm_krylov::FINISHED) return fail(UHM_EINVAL, "the solve has not finished");
  const int64_t n = K->n;
  const int r = K->r;
  if (X) {
    if (ldx < n) return fail(UHM_EINVAL, "leading dimension smaller than n");
    hipLaunchKernelGGL(k_g_add, dim3(nblk(n * r)), dim3(kGB), 0, K->s, K->xacc.p, n, r, static_cast<cd*>(X), ldx, 1);
    UHM_HIP(hipStreamSynchronize(K->s));
  }
  int conv = 0;
  double worst = 0.0;
  for (int c = 0; c < r; ++c) {
    const double rel = K->bn[c] > 0.0 ? K->rn[c] / K->bn[c] : 0.0;
    worst = std::max(worst, rel);
    conv += rel <= K->tol;
  }
  if (info) {
    info->iterations = K->iters;
    info->restarts = K->restarts;
    info->refinements = K->mixed ? K->refinements : 0;
    info->converged = conv;
    info->rel_residual = worst;
    info->seconds_total = 0.0;
    info->seconds_products = 0.0;
    info->seconds_arnoldi = K->t_arn;
    UHM_HIP(hipMemcpyAsync(K->W.hreorth.p, K->W.reorth.p, sizeof(unsigned long long), hipMemcpyDeviceToHost, K->s));
    UHM_HIP(hipStreamSynchronize(K->s));
    info->second_passes = (int64_t)K->W.hreorth.p[0];
  }
  return conv == r ? UHM_OK : fail(UHM_ENOCONV, "iteration limit reached before the tolerance");
}

void uhm_krylov_free(uhm_krylov* K) { delete K; }

// One step of many solves: their pending products, one multi-column product per
// (operator, precision) group, then every solve advances.  Returns the number of solves
// still running (>= 0) or an error code.
int uhm_krylov_step(uhm_krylov* const* ks, uhm_op* const* high, uhm_op* const* low, int32_t count, void* hip_stream) {
  if (count < 0 || (count > 0 && (!ks || !high))) return fail(UHM_EINVAL, "null argument");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  struct Item {
    int32_t k;
    int kind;
    const cd* in;
    cd* out;
  };
  std::map<std::pair<uhm_op*, int>, std::vector<Item>> groups;
  for (int32_t k = 0; k < count; ++k) {
    uhm_krylov* K = ks[k];
    if (!K) return fail(UHM_EINVAL, "null solve");
    if (K->req == UHM_KRYLOV_DONE) continue;
    uhm_op* A = K->req == UHM_KRYLOV_PRODUCT_HIGH ? high[k] : (low ? low[k] : nullptr);
    if (!A || A->n != K->n || A->kind != 0) return fail(UHM_EINVAL, "missing or mismatched operator for a solve");
    if (!A->lp && !is_c128(A->storage))
      return fail(UHM_ENOTSUP, "uhm_krylov_step takes complex128 or many-RHS low-precision operators");
    const bool want_hi = K->req == UHM_KRYLOV_PRODUCT_HIGH;
    const bool is_hi = is_c128(A->storage);
    if (want_hi != is_hi) return fail(UHM_EINVAL, "operator precision does not match the request");
    groups[{A, K->req}].push_back({k, K->req, static_cast<const cd*>(K->req_in), static_cast<cd*>(K->req_out)});
  }
  int rc;
  // products run on s: work a solve queued earlier on its own stream must be complete
  bool all_on_s = true;
  std::vector<hipStream_t> other;
  for (int32_t k = 0; k < count; ++k)
    if (ks[k]->s != s) {
      all_on_s = false;
      if (std::find(other.begin(), other.end(), ks[k]->s) == other.end()) other.push_back(ks[k]->s);
    }
  for (hipStream_t o : other) UHM_HIP(hipStreamSynchronize(o));
  StepScratch& ss = step_scratch();
  std::lock_guard<std::mutex> lock(ss.mu);
  // products of up to 64 columns (whole solves) per operator and precision
  struct Chunk {
    uhm_op* A;
    bool hi;
    const Item* items;
    size_t cnt;
    int cols;
    size_t poff;  // first x pointer in the step's pointer array (y pointers follow the x ones)
  };
  std::vector<Chunk> chunks;
  size_t nptr = 0;
  for (auto& gkv : groups) {
    const std::vector<Item>& items = gkv.second;
    size_t a = 0;
    while (a < items.size()) {
      int cols = 0;
      size_t b = a;
      while (b < items.size() && (cols == 0 || cols + ks[items[b].k]->r <= 64)) cols += ks[items[b++].k]->r;
      Chunk c{gkv.first.first, gkv.first.second == UHM_KRYLOV_PRODUCT_HIGH, &items[a], b - a, cols, nptr};
      if (c.A->lp) nptr += 2 * (size_t)cols;
      chunks.push_back(c);
      a = b;
    }
  }
  // many-RHS operators read and write the solves' vectors through column pointers
  if (nptr > 0) {
    if (ss.pev_recorded) UHM_HIP(hipEventSynchronize(ss.pev));
    if (!ss.pev) UHM_HIP(hipEventCreateWithFlags(&ss.pev, hipEventDisableTiming));
    if (nptr > ss.pcap) {
      if (ss.pdev) (void)hipFree(ss.pdev);
      if (ss.phost) (void)hipHostFree(ss.phost);
      ss.pdev = ss.phost = nullptr;
      const size_t cap = std::max(nptr, 2 * ss.pcap + 1024);
      ss.pcap = 0;
      UHM_HIP(hipMalloc(reinterpret_cast<void**>(&ss.pdev), sizeof(cd*) * cap));
      UHM_HIP(hipHostMalloc(reinterpret_cast<void**>(&ss.phost), sizeof(cd*) * cap, hipHostMallocDefault));
      ss.pcap = cap;
    }
    for (const Chunk& c : chunks) {
      if (!c.A->lp) continue;
      size_t q = c.poff;
      for (size_t t = 0; t < c.cnt; ++t)
        for (int j = 0; j < ks[c.items[t].k]->r; ++j) ss.phost[q++] = c.items[t].in + (int64_t)j * c.A->n;
      for (size_t t = 0; t < c.cnt; ++t)
        for (int j = 0; j < ks[c.items[t].k]->r; ++j) ss.phost[q++] = c.items[t].out + (int64_t)j * c.A->n;
    }
    UHM_HIP(hipMemcpyAsync(ss.pdev, ss.phost, sizeof(cd*) * nptr, hipMemcpyHostToDevice, s));
    UHM_HIP(hipEventRecord(ss.pev, s));
    ss.pev_recorded = true;
  }
  // many-RHS products in shared stage launches: one call per (storage, column blocks,
  // chunk number of the operator), every operator at most once per call
  {
    std::map<std::tuple<int, int, int>, std::vector<const Chunk*>> sets;
    std::map<uhm_op*, int> seen;
    for (const Chunk& c : chunks)
      if (c.A->lp) sets[{c.A->storage, (c.cols + 15) / 16, seen[c.A]++}].push_back(&c);
    for (auto& kv : sets) {
      std::vector<uhm_op*> ops;
      std::vector<const cd* const*> xc;
      std::vector<cd* const*> yc;
      std::vector<int32_t> nc;
      for (const Chunk* c : kv.second) {
        ops.push_back(c->A);
        xc.push_back(ss.pdev + c->poff);
        yc.push_back(const_cast<cd* const*>(ss.pdev + c->poff + c->cols));
        nc.push_back(c->cols);
      }
      if ((rc = lowp_step_products(ops.data(), xc.data(), yc.data(), nc.data(), (int32_t)ops.size(), s))) return rc;
    }
  }
  for (const Chunk& c : chunks) {
    uhm_op* A = c.A;
    const int64_t n = A->n;
    if (A->lp) continue;
    // single-RHS storage: pack the columns, multiply, unpack
    const int64_t need = 16 * n * c.cols;
    if (A->stage_bytes < need) {
      if ((rc = A->stage_in.alloc(need)) || (rc = A->stage_out.alloc(need))) {
        A->stage_bytes = 0;
        return rc;
      }
      A->stage_bytes = need;
    }
    int c0 = 0;
    for (size_t t = 0; t < c.cnt; ++t) {
      const int r = ks[c.items[t].k]->r;
      UHM_HIP(hipMemcpyAsync(reinterpret_cast<cd*>(A->stage_in.p) + (int64_t)c0 * n, c.items[t].in,
                             sizeof(cd) * (size_t)(n * r), hipMemcpyDeviceToDevice, s));
      c0 += r;
    }
    if ((rc = uhm_matvec(A, A->stage_in.p, n, A->stage_out.p, n, c.cols, s))) return rc;
    c0 = 0;
    for (size_t t = 0; t < c.cnt; ++t) {
      const int r = ks[c.items[t].k]->r;
      UHM_HIP(hipMemcpyAsync(c.items[t].out, reinterpret_cast<cd*>(A->stage_out.p) + (int64_t)c0 * n,
                             sizeof(cd) * (size_t)(n * r), hipMemcpyDeviceToDevice, s));
      c0 += r;
    }
  }
  if (!all_on_s) UHM_HIP(hipStreamSynchronize(s));
  // Arnoldi steps of all solves: one launch per kernel over all of them on s, one
  // synchronisation, then the host halves.  Other phases advance one by one.
  std::vector<uhm_krylov*> iter;
  for (int32_t k = 0; k < count; ++k) {
    uhm_krylov* K = ks[k];
    if (K->req != UHM_KRYLOV_DONE && K->phase == uhm_krylov::ITER) iter.push_back(K);
  }
  if (!iter.empty()) {
    const auto t0 = Clock::now();
    ManyLayout Lo{};
    if ((rc = arnoldi_issue_many(iter, s, ss, Lo))) return rc;
    UHM_HIP(hipStreamSynchronize(s));
    if ((rc = arnoldi_finish_many(iter, ss, Lo))) return rc;
    const double dt = std::chrono::duration<double>(Clock::now() - t0).count() / (double)iter.size();
    for (uhm_krylov* K : iter) K->t_arn += dt;
  }
  int running = 0;
  for (int32_t k = 0; k < count; ++k) {
    uhm_krylov* K = ks[k];
    if (K->req == UHM_KRYLOV_DONE) continue;
    if (std::find(iter.begin(), iter.end(), K) == iter.end() && (rc = uhm_krylov_advance(K))) return rc;
    running += K->req != UHM_KRYLOV_DONE;
  }
  return running;
}

int uhm_solve_gmres(uhm_op* op, uhm_op* inner, const void* B, int64_t ldb, void* X, int64_t ldx, int32_t nrhs,
                    double tol, const uhm_gmres_opts* opts, uhm_gmres_info* info, void* hip_stream) {
  if (!op || !B || !X) return fail(UHM_EINVAL, "null argument");
  if (!is_c128(op->storage) || op->kind != 0)
    return fail(UHM_EINVAL, "the residual operator must be a complex128 UH-matrix");
  if (inner && (is_c128(inner->storage) || inner->kind != 0 || inner->n != op->n))
    return fail(UHM_EINVAL, "the inner operator must be a low-precision form of the same size");
  if (nrhs < 1 || ldx < op->n) return fail(UHM_EINVAL, "bad nrhs or leading dimension");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const auto t0 = Clock::now();
  uhm_krylov* K = nullptr;
  int rc = uhm_krylov_create(op->n, nrhs, B, ldb, tol, inner != nullptr, opts, hip_stream, &K);
  if (rc) return rc;
  std::unique_ptr<uhm_krylov> hold(K);
  // product buffers for the low-precision operator
  DevArray<cf> in32, out32;
  const int64_t nq = op->n * (int64_t)nrhs;
  if (inner && ((rc = in32.alloc(nq)) || (rc = out32.alloc(nq)))) return rc;
  // GPU time of the products from events around them, read two products late so that the
  // host never waits for work it has just issued
  struct Events {
    hipEvent_t e[2][2] = {};
    ~Events() {
      for (auto& pr : e)
        for (hipEvent_t x : pr)
          if (x) (void)hipEventDestroy(x);
    }
  } pe;
  for (auto& pr : pe.e)
    for (hipEvent_t& x : pr) UHM_HIP(hipEventCreate(&x));
  double t_prod = 0.0;
  int64_t np = 0;
  auto take = [&](int slot) -> int {
    float ms = 0.f;
    UHM_HIP(hipEventSynchronize(pe.e[slot][1]));
    UHM_HIP(hipEventElapsedTime(&ms, pe.e[slot][0], pe.e[slot][1]));
    t_prod += 1e-3 * ms;
    return UHM_OK;
  };
  while (true) {
    const void* in = nullptr;
    void* out = nullptr;
    const int what = uhm_krylov_next(K, &in, &out);
    if (what == UHM_KRYLOV_DONE) break;
    const int slot = (int)(np & 1);
    if (np >= 2 && (rc = take(slot))) return rc;
    UHM_HIP(hipEventRecord(pe.e[slot][0], s));
    if (what == UHM_KRYLOV_PRODUCT_HIGH) {
      rc = uhm_matvec(op, in, op->n, out, op->n, nrhs, s);
    } else {
      hipLaunchKernelGGL(k_g_to32, dim3(nblk(nq)), dim3(kGB), 0, s, static_cast<const cd*>(in), nq, in32.p);
      rc = uhm_matvec(inner, in32.p, op->n, out32.p, op->n, nrhs, s);
      if (rc == UHM_OK) hipLaunchKernelGGL(k_g_to64, dim3(nblk(nq)), dim3(kGB), 0, s, out32.p, nq, static_cast<cd*>(out));
    }
    if (rc) return rc;
    UHM_HIP(hipEventRecord(pe.e[slot][1], s));
    ++np;
    if ((rc = uhm_krylov_advance(K))) return rc;
  }
  for (int64_t q = std::max<int64_t>(0, np - 2); q < np; ++q)
    if ((rc = take((int)(q & 1)))) return rc;
  rc = uhm_krylov_result(K, X, ldx, info);
  if (info) {
    info->seconds_total = std::chrono::duration<double>(Clock::now() - t0).count();
    info->seconds_products = t_prod;
    // everything else: orthogonalisation, least-squares updates, residuals, control
    info->seconds_arnoldi = std::max(0.0, info->seconds_total - t_prod);
  }
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return fail(UHM_EHIP, std::string("gmres kernels: ") + hipGetErrorString(he));
  return rc;
}

}  // extern "C"
