// Batched restarted GMRES(m) and mixed-precision GMRES with iterative refinement.
//
// Every right-hand side has its own Krylov space; all of them advance in lockstep so that
// each Arnoldi step is one batched product with the operator (uhm_matvec over nrhs
// columns) plus batched FP64 kernels:
//   dots     h_i = V_i^* w for i <= j (classical Gram-Schmidt), per column,
//   update   w -= sum_i V_i h_i, with the partial sums of ||w||^2,
//   scale    V_{j+1} = w / ||w||,
// and Gram-Schmidt is applied twice.  The reductions are two-pass over fixed row chunks
// (deterministic).  The (m+1) x m Hessenberg matrices, the Givens rotations and the small
// triangular solves are done on the host in FP64 from the few numbers each step produces.
//
// With an inner operator (complex64 or bf16 pairs) the solve is iterative refinement: the
// residual r = b - A x is formed with the FP64 operator, an inner GMRES(m) whose products
// use the low-precision operator (vectors converted to complex64 for the product and back)
// reduces it by inner_tol, and x += d.
#include "uhm_internal.h"

#include <chrono>
#include <cmath>
#include <complex>

namespace uhm_detail {
namespace {

using cf = float2;
constexpr int kGB = 256;      // threads per block
constexpr int kGRows = 2048;  // rows per block in the batched reductions

__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
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

// part[((i * r) + c) * nch + ch] = sum over the chunk's rows of conj(V_i[row, c]) w[row, c]
__global__ __launch_bounds__(kGB) void k_g_dots(const cd* __restrict__ V, int64_t vstride, int nvec,
                                                const cd* __restrict__ w, int64_t n, int r, int nch,
                                                cd* __restrict__ part) {
  __shared__ double sh[2 * kGB / 64];
  const int ch = blockIdx.x, c = blockIdx.y;
  const int64_t r0 = (int64_t)ch * kGRows;
  const int64_t r1 = min(n, r0 + kGRows);
  constexpr int PER = kGRows / kGB;
  cd wv[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int64_t row = r0 + threadIdx.x + (int64_t)q * kGB;
    wv[q] = row < r1 ? w[(int64_t)c * n + row] : make_double2(0.0, 0.0);
  }
  for (int i = 0; i < nvec; ++i) {
    const cd* vi = V + (int64_t)i * vstride + (int64_t)c * n;
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int64_t row = r0 + threadIdx.x + (int64_t)q * kGB;
      if (row < r1) {
        const cd v = vi[row];
        re = fma(v.x, wv[q].x, fma(v.y, wv[q].y, re));
        im = fma(v.x, wv[q].y, fma(-v.y, wv[q].x, im));
      }
    }
    double sr, si;
    block_sum2(re, im, sh, sr, si);
    if (threadIdx.x == 0) part[((int64_t)i * r + c) * nch + ch] = make_double2(sr, si);
  }
}

// out[q] = sum_ch part[q * nch + ch]
__global__ __launch_bounds__(kGB) void k_g_reduce(const cd* __restrict__ part, int nch, int64_t nq, cd* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * kGB + threadIdx.x;
  if (q >= nq) return;
  double re = 0.0, im = 0.0;
  for (int ch = 0; ch < nch; ++ch) {
    const cd v = part[q * nch + ch];
    re += v.x;
    im += v.y;
  }
  out[q] = make_double2(re, im);
}

// w[:, c] -= sum_i V_i[:, c] h[i * r + c]; nrm[c * nch + ch] = partial ||w_new||^2
__global__ __launch_bounds__(kGB) void k_g_update(const cd* __restrict__ V, int64_t vstride, int nvec,
                                                  const cd* __restrict__ h, cd* __restrict__ w, int64_t n, int r,
                                                  int nch, double* __restrict__ nrm) {
  __shared__ double sh[2 * kGB / 64];
  const int ch = blockIdx.x, c = blockIdx.y;
  const int64_t r0 = (int64_t)ch * kGRows;
  const int64_t r1 = min(n, r0 + kGRows);
  double acc = 0.0;
  for (int64_t row = r0 + threadIdx.x; row < r1; row += kGB) {
    cd a = w[(int64_t)c * n + row];
    for (int i = 0; i < nvec; ++i) {
      const cd v = V[(int64_t)i * vstride + (int64_t)c * n + row];
      const cd hi = h[(int64_t)i * r + c];
      a.x -= v.x * hi.x - v.y * hi.y;
      a.y -= v.x * hi.y + v.y * hi.x;
    }
    w[(int64_t)c * n + row] = a;
    acc += a.x * a.x + a.y * a.y;
  }
  double s, dummy;
  block_sum2(acc, 0.0, sh, s, dummy);
  if (threadIdx.x == 0) nrm[(int64_t)c * nch + ch] = s;
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

struct Work {
  int64_t n = 0;
  int r = 0, m = 0, nch = 0;
  DevArray<cd> V, w, t, d, part, hbuf, ybuf;
  DevArray<double> nrm, nrm_out;
  DevArray<cf> x32, y32;
  double t_prod = 0.0, t_arn = 0.0;
};

int alloc_work(Work& W, int64_t n, int r, int m, bool lowp) {
  W.n = n;
  W.r = r;
  W.m = m;
  W.nch = (int)((n + kGRows - 1) / kGRows);
  int rc;
  if ((rc = W.V.alloc((int64_t)(m + 1) * n * r)) || (rc = W.w.alloc(n * r)) || (rc = W.t.alloc(n * r)) ||
      (rc = W.d.alloc(n * r)) || (rc = W.part.alloc((int64_t)(m + 1) * r * W.nch)) ||
      (rc = W.hbuf.alloc((int64_t)(m + 1) * r)) || (rc = W.ybuf.alloc((int64_t)(m + 1) * r)) ||
      (rc = W.nrm.alloc((int64_t)r * W.nch)) || (rc = W.nrm_out.alloc(r)))
    return rc;
  if (lowp && ((rc = W.x32.alloc(n * r)) || (rc = W.y32.alloc(n * r)))) return rc;
  return UHM_OK;
}

// y = A x for contiguous n x r FP64 arrays, with A in any storage.
int apply(uhm_op* A, Work& W, const cd* x, cd* y, hipStream_t s) {
  const auto t0 = Clock::now();
  int rc;
  if (A->storage == UHM_C128 || A->storage == UHM_C128_MULTI) {
    rc = uhm_matvec(A, x, W.n, y, W.n, W.r, s);
  } else {
    const int64_t nq = W.n * W.r;
    hipLaunchKernelGGL(k_g_to32, dim3(nblk(nq)), dim3(kGB), 0, s, x, nq, W.x32.p);
    rc = uhm_matvec(A, W.x32.p, W.n, W.y32.p, W.n, W.r, s);
    if (rc == UHM_OK) hipLaunchKernelGGL(k_g_to64, dim3(nblk(nq)), dim3(kGB), 0, s, W.y32.p, nq, y);
  }
  if (rc) return rc;
  UHM_HIP(hipStreamSynchronize(s));
  W.t_prod += std::chrono::duration<double>(Clock::now() - t0).count();
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

// Restarted GMRES(m) for A d = rhs (contiguous n x r), from d = 0 (W.d), until
// ||rhs - A d_c|| <= rtol_c (per column) or `budget` Krylov iterations in total.
int gmres_cycles(uhm_op* A, Work& W, const cd* rhs, const std::vector<double>& rtol, int budget, int& iters,
                 int& restarts, std::vector<char>& done, hipStream_t s) {
  const int r = W.r, m = W.m;
  const int64_t n = W.n, vstride = n * r;
  int rc;
  UHM_HIP(hipMemsetAsync(W.d.p, 0, sizeof(cd) * (size_t)(n * r), s));
  UHM_HIP(hipMemcpyAsync(W.t.p, rhs, sizeof(cd) * (size_t)(n * r), hipMemcpyDeviceToDevice, s));
  bool first = true;
  std::vector<double> beta;
  std::vector<C> H((size_t)(m + 1) * m * r), g((size_t)(m + 1) * r), cs((size_t)m * r), sn((size_t)m * r);
  std::vector<cd> hh((size_t)(m + 1) * r), hp;
  std::vector<int> jc(r);
  std::vector<double> sc(r), hn(r);
  while (true) {
    if ((rc = norms(W, W.t.p, beta, s))) return rc;
    bool all = true;
    for (int c = 0; c < r; ++c) {
      done[c] = beta[c] <= rtol[c];
      all = all && done[c];
    }
    if (all || iters >= budget) return UHM_OK;
    if (!first) ++restarts;
    first = false;
    for (int c = 0; c < r; ++c) sc[c] = beta[c] > 0.0 ? 1.0 / beta[c] : 0.0;
    UHM_HIP(hipMemcpyAsync(W.nrm_out.p, sc.data(), sizeof(double) * r, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_g_scale, dim3(nblk(n * r)), dim3(kGB), 0, s, W.t.p, W.nrm_out.p, n, r, W.V.p);
    std::fill(g.begin(), g.end(), C(0.0));
    std::vector<char> active(r);
    for (int c = 0; c < r; ++c) {
      g[(size_t)c * (m + 1)] = C(beta[c]);
      jc[c] = 0;
      active[c] = !done[c];
    }
    int j = 0;
    for (; j < m && iters < budget; ++j) {
      if ((rc = apply(A, W, W.V.p + (int64_t)j * vstride, W.w.p, s))) return rc;
      ++iters;
      const auto ta = Clock::now();
      hp.resize((size_t)(j + 1) * r);
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(k_g_dots, dim3(W.nch, r), dim3(kGB), 0, s, W.V.p, vstride, j + 1, W.w.p, n, r, W.nch,
                           W.part.p);
        hipLaunchKernelGGL(k_g_reduce, dim3(nblk((int64_t)(j + 1) * r)), dim3(kGB), 0, s, W.part.p, W.nch,
                           (int64_t)(j + 1) * r, W.hbuf.p);
        hipLaunchKernelGGL(k_g_update, dim3(W.nch, r), dim3(kGB), 0, s, W.V.p, vstride, j + 1, W.hbuf.p, W.w.p, n, r,
                           W.nch, W.nrm.p);
        UHM_HIP(hipMemcpyAsync(hp.data(), W.hbuf.p, sizeof(cd) * hp.size(), hipMemcpyDeviceToHost, s));
        UHM_HIP(hipStreamSynchronize(s));
        for (size_t q = 0; q < hp.size(); ++q) {
          if (pass == 0) {
            hh[q] = hp[q];
          } else {
            hh[q].x += hp[q].x;
            hh[q].y += hp[q].y;
          }
        }
      }
      hipLaunchKernelGGL(k_g_norm, dim3((r + 63) / 64), dim3(64), 0, s, W.nrm.p, W.nch, r, W.nrm_out.p);
      UHM_HIP(hipMemcpyAsync(hn.data(), W.nrm_out.p, sizeof(double) * r, hipMemcpyDeviceToHost, s));
      UHM_HIP(hipStreamSynchronize(s));
      bool all_done = true;
      for (int c = 0; c < r; ++c) {
        sc[c] = 0.0;
        if (!active[c]) continue;
        C* col = &H[((size_t)c * m + j) * (m + 1)];
        for (int i = 0; i <= j; ++i) col[i] = C(hh[(size_t)i * r + c].x, hh[(size_t)i * r + c].y);
        col[j + 1] = C(hn[c]);
        sc[c] = hn[c] > 1e-300 ? 1.0 / hn[c] : 0.0;
        for (int i = 0; i < j; ++i) {
          const C a = col[i], b = col[i + 1];
          const C ci = cs[(size_t)c * m + i], si = sn[(size_t)c * m + i];
          col[i] = std::conj(ci) * a + std::conj(si) * b;
          col[i + 1] = -si * a + ci * b;
        }
        const C a = col[j], b = col[j + 1];
        const double den = std::sqrt(std::norm(a) + std::norm(b));
        C cj(1.0), sj(0.0);
        if (den > 0.0) {
          cj = a / den;
          sj = b / den;
        }
        cs[(size_t)c * m + j] = cj;
        sn[(size_t)c * m + j] = sj;
        col[j] = std::conj(cj) * a + std::conj(sj) * b;
        col[j + 1] = C(0.0);
        C* gc = &g[(size_t)c * (m + 1)];
        const C gj = gc[j];
        gc[j] = std::conj(cj) * gj;
        gc[j + 1] = -sj * gj;
        jc[c] = j + 1;
        if (std::abs(gc[j + 1]) <= rtol[c] || hn[c] <= 1e-300) active[c] = 0;
        all_done = all_done && !active[c];
      }
      UHM_HIP(hipMemcpyAsync(W.nrm_out.p, sc.data(), sizeof(double) * r, hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_g_scale, dim3(nblk(n * r)), dim3(kGB), 0, s, W.w.p, W.nrm_out.p, n, r,
                         W.V.p + (int64_t)(j + 1) * vstride);
      UHM_HIP(hipStreamSynchronize(s));
      W.t_arn += std::chrono::duration<double>(Clock::now() - ta).count();
      if (all_done) {
        ++j;
        break;
      }
    }
    // y_c = R_c^{-1} g_c (back substitution), d += V y
    const auto ta = Clock::now();
    const int jm = j;
    if (jm > 0) {
      std::vector<cd> yv((size_t)jm * r, make_double2(0.0, 0.0));
      for (int c = 0; c < r; ++c) {
        const int k = jc[c];
        const C* Hc = &H[(size_t)c * m * (m + 1)];
        const C* gc = &g[(size_t)c * (m + 1)];
        std::vector<C> y(k);
        for (int i = k - 1; i >= 0; --i) {
          C acc = gc[i];
          for (int q = i + 1; q < k; ++q) acc -= Hc[(size_t)q * (m + 1) + i] * y[q];
          const C dgl = Hc[(size_t)i * (m + 1) + i];
          y[i] = std::abs(dgl) > 0.0 ? acc / dgl : C(0.0);
        }
        for (int i = 0; i < k; ++i) yv[(size_t)i * r + c] = make_double2(y[i].real(), y[i].imag());
      }
      UHM_HIP(hipMemcpyAsync(W.ybuf.p, yv.data(), sizeof(cd) * yv.size(), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_g_combine, dim3(nblk(n * r)), dim3(kGB), 0, s, W.V.p, vstride, jm, W.ybuf.p, W.d.p, n, n, r);
    }
    UHM_HIP(hipStreamSynchronize(s));
    W.t_arn += std::chrono::duration<double>(Clock::now() - ta).count();
    // residual for the next cycle: t = rhs - A d
    if ((rc = apply(A, W, W.d.p, W.w.p, s))) return rc;
    hipLaunchKernelGGL(k_g_sub, dim3(nblk(n * r)), dim3(kGB), 0, s, rhs, n, W.w.p, n, r, W.t.p);
  }
}

}  // namespace
}  // namespace uhm_detail

using namespace uhm_detail;

extern "C" int uhm_solve_gmres(uhm_op* op, uhm_op* inner, const void* B, int64_t ldb, void* X, int64_t ldx, int32_t nrhs,
                               double tol, const uhm_gmres_opts* opts, uhm_gmres_info* info, void* hip_stream) {
  if (!op || !B || !X) return fail(UHM_EINVAL, "null argument");
  if ((op->storage != UHM_C128 && op->storage != UHM_C128_MULTI) || op->kind != 0)
    return fail(UHM_EINVAL, "the residual operator must be a complex128 UH-matrix");
  if (inner && (inner->storage == UHM_C128 || inner->storage == UHM_C128_MULTI || inner->n != op->n))
    return fail(UHM_EINVAL, "the inner operator must be a low-precision form of the same size");
  if (nrhs < 1 || ldb < op->n || ldx < op->n || !(tol > 0.0)) return fail(UHM_EINVAL, "bad nrhs, leading dimension or tol");
  uhm_gmres_opts o{50, 2000, 30, 1e-4};
  if (opts) o = *opts;
  if (o.restart < 1 || o.max_iterations < 1 || o.max_refinements < 1 || !(o.inner_tol > 0.0) || o.inner_tol >= 1.0)
    return fail(UHM_EINVAL, "bad GMRES options");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const auto t0 = Clock::now();
  const int64_t n = op->n;
  const int r = nrhs;
  Work W;
  int rc = alloc_work(W, n, r, o.restart, inner != nullptr);
  if (rc) return rc;
  DevArray<cd> Bc, xacc, res;
  if ((rc = Bc.alloc(n * r)) || (rc = res.alloc(n * r))) return rc;
  hipLaunchKernelGGL(k_g_copy_strided, dim3(nblk(n * r)), dim3(kGB), 0, s, static_cast<const cd*>(B), ldb, n, r, Bc.p);
  std::vector<double> bn, rn;
  if ((rc = norms(W, Bc.p, bn, s))) return rc;
  int iters = 0, restarts = 0, refinements = 0;
  std::vector<char> done(r, 0);
  cd* Xd = static_cast<cd*>(X);
  if (!inner) {
    std::vector<double> rtol(r);
    for (int c = 0; c < r; ++c) rtol[c] = tol * bn[c];
    if ((rc = gmres_cycles(op, W, Bc.p, rtol, o.max_iterations, iters, restarts, done, s))) return rc;
    hipLaunchKernelGGL(k_g_add, dim3(nblk(n * r)), dim3(kGB), 0, s, W.d.p, n, r, Xd, ldx, 1);
    if ((rc = apply(op, W, W.d.p, W.w.p, s))) return rc;
    hipLaunchKernelGGL(k_g_sub, dim3(nblk(n * r)), dim3(kGB), 0, s, Bc.p, n, W.w.p, n, r, res.p);
    if ((rc = norms(W, res.p, rn, s))) return rc;
  } else {
    if ((rc = xacc.alloc(n * r))) return rc;
    UHM_HIP(hipMemsetAsync(xacc.p, 0, sizeof(cd) * (size_t)(n * r), s));
    UHM_HIP(hipMemcpyAsync(res.p, Bc.p, sizeof(cd) * (size_t)(n * r), hipMemcpyDeviceToDevice, s));
    if ((rc = norms(W, res.p, rn, s))) return rc;
    while (true) {
      bool all = true;
      for (int c = 0; c < r; ++c) all = all && rn[c] <= tol * bn[c];
      if (all || refinements >= o.max_refinements || iters >= o.max_iterations) break;
      std::vector<double> rtol(r);
      for (int c = 0; c < r; ++c) rtol[c] = o.inner_tol * rn[c];
      if ((rc = gmres_cycles(inner, W, res.p, rtol, o.max_iterations, iters, restarts, done, s))) return rc;
      ++refinements;
      hipLaunchKernelGGL(k_g_add, dim3(nblk(n * r)), dim3(kGB), 0, s, W.d.p, n, r, xacc.p, n, 0);
      if ((rc = apply(op, W, xacc.p, W.w.p, s))) return rc;
      hipLaunchKernelGGL(k_g_sub, dim3(nblk(n * r)), dim3(kGB), 0, s, Bc.p, n, W.w.p, n, r, res.p);
      if ((rc = norms(W, res.p, rn, s))) return rc;
    }
    hipLaunchKernelGGL(k_g_add, dim3(nblk(n * r)), dim3(kGB), 0, s, xacc.p, n, r, Xd, ldx, 1);
  }
  UHM_HIP(hipStreamSynchronize(s));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(UHM_EHIP, std::string("gmres kernels: ") + hipGetErrorString(e));
  int conv = 0;
  double worst = 0.0;
  for (int c = 0; c < r; ++c) {
    const double rel = bn[c] > 0.0 ? rn[c] / bn[c] : 0.0;
    worst = std::max(worst, rel);
    conv += rel <= tol;
  }
  if (info) {
    info->iterations = iters;
    info->restarts = restarts;
    info->refinements = refinements;
    info->converged = conv;
    info->rel_residual = worst;
    info->seconds_total = std::chrono::duration<double>(Clock::now() - t0).count();
    info->seconds_products = W.t_prod;
    info->seconds_arnoldi = W.t_arn;
  }
  return conv == r ? UHM_OK : fail(UHM_ENOCONV, "iteration limit reached before the tolerance");
}
