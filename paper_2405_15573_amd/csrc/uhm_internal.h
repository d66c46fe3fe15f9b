// Internal declarations shared by the translation units of libuhm.so.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "uhm.h"

namespace uhm_detail {

extern thread_local std::string g_err;

inline int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define UHM_HIP(call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? UHM_ENOMEM : UHM_EHIP,                         \
                  std::string(#call) + ": " + hipGetErrorString(e_));                       \
    }                                                                                        \
  } while (0)

constexpr int kLeafMax = 64;     // leaf size bound: one lane per leaf row
constexpr int kTile = 64;        // forward-panel tile width (one lane per column)
constexpr int kRowChunk = 64;    // coupling row chunk (one lane per row)
constexpr int kCoupCols = 256;   // coupling columns per wavefront tile
constexpr int kFwdWaves = 4;
constexpr int kBwdWaves = 4;
constexpr int kBwdChunk = 512;   // z entries staged in LDS per round
constexpr int kCoupWaves = 4;

using cd = double2;
struct CoupTile {
  int64_t s_base;     // element offset of the tile's first column
  int32_t h;          // rows in the chunk (<= 64)
  int32_t ncols;      // columns in the tile
  int32_t first_blk;  // index into the block list of the tile's first column
  int32_t first_col;  // column within that block
};

// Coupling tile of the symmetric storage form: a column range of one row chunk of
// [S_b1 S_b2 ...] (stored blocks of one row cluster), read once for S_b u_sigma and for
// S_b^T u_tau.
struct SymTile {
  int64_t s_base;  // element offset of the tile's first column
  int64_t t_base;  // transposed-partial index of the tile's first column
  int32_t c_base;  // index into the column-source table of the tile's first column
  int32_t h;       // rows in the chunk (<= 64)
  int32_t ncols;   // columns in the tile
  int32_t x_row;   // rank-space index of the chunk's first row
};

// A tile of the first step of factored couplings: wj (<= 64) columns of the panel
// [S_{Y,b1} S_{Y,b2} ...] of one column cluster sigma (l_sigma rows, row-major tile).
struct FacTile {
  int64_t f_base;  // element offset of the tile
  int32_t rows;    // l_sigma
  int32_t wj;      // columns in the tile
  int32_t x_row;   // rank-space index of u_sigma
  int32_t t_out;   // index of the tile's first result in the coupling source vector
};

template <class T>
struct DevArray {
  T* p = nullptr;
  int64_t n = 0;
  ~DevArray() {
    if (p) (void)hipFree(p);
  }
  // (Re)allocates; the previous contents are released.
  int alloc(int64_t count) {
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
    n = count;
    if (count == 0) return UHM_OK;
    hipError_t e = hipMalloc(&p, sizeof(T) * (size_t)count);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(e == hipErrorOutOfMemory ? UHM_ENOMEM : UHM_EHIP,
                  std::string("hipMalloc(") + std::to_string(sizeof(T) * (size_t)count) + " B): " + hipGetErrorString(e));
    }
    return UHM_OK;
  }
  int upload(const std::vector<T>& v, hipStream_t s) {
    int rc = alloc((int64_t)v.size());
    if (rc) return rc;
    if (!v.empty()) UHM_HIP(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
    return UHM_OK;
  }
  size_t bytes() const { return sizeof(T) * (size_t)n; }
};

// Streams host-packed data into a device array through two pinned staging buffers.
template <class E>
struct StagerT {
  E* dev = nullptr;
  int64_t total = 0, written = 0;
  hipStream_t s = nullptr;
  E* host[2] = {nullptr, nullptr};
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool pending[2] = {false, false};
  int64_t cap = 0, fill = 0;
  int cur = 0;
  int err = UHM_OK;

  int init(E* d, int64_t tot, hipStream_t st) {
    dev = d;
    total = tot;
    s = st;
    cap = std::max<int64_t>(1, std::min<int64_t>(tot, (int64_t)(64 << 20) / (int64_t)sizeof(E)));
    for (int b = 0; b < 2; ++b) {
      UHM_HIP(hipHostMalloc(reinterpret_cast<void**>(&host[b]), sizeof(E) * (size_t)cap, hipHostMallocDefault));
      UHM_HIP(hipEventCreateWithFlags(&ev[b], hipEventDisableTiming));
    }
    return UHM_OK;
  }
  // Room for k <= cap elements in the current staging buffer.
  E* span(int64_t k) {
    if (fill + k > cap) flush();
    E* r = host[cur] + fill;
    fill += k;
    return r;
  }
  void flush() {
    if (fill == 0 || err) return;
    if (written + fill > total) {
      err = fail(UHM_EINVAL, "internal: staged more elements than allocated");
      return;
    }
    hipError_t e = hipMemcpyAsync(dev + written, host[cur], sizeof(E) * (size_t)fill, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(ev[cur], s);
    if (e != hipSuccess) {
      err = fail(UHM_EHIP, std::string("staged copy: ") + hipGetErrorString(e));
      return;
    }
    pending[cur] = true;
    written += fill;
    fill = 0;
    cur ^= 1;
    if (pending[cur]) {
      e = hipEventSynchronize(ev[cur]);
      pending[cur] = false;
      if (e != hipSuccess) err = fail(UHM_EHIP, std::string("staged copy sync: ") + hipGetErrorString(e));
    }
  }
  int finish() {
    flush();
    for (int b = 0; b < 2; ++b)
      if (pending[b]) {
        (void)hipEventSynchronize(ev[b]);
        pending[b] = false;
      }
    if (!err && written != total) err = fail(UHM_EINVAL, "internal: staged element count mismatch");
    return err;
  }
  ~StagerT() {
    for (int b = 0; b < 2; ++b) {
      if (pending[b]) (void)hipEventSynchronize(ev[b]);
      if (host[b]) (void)hipHostFree(host[b]);
      if (ev[b]) (void)hipEventDestroy(ev[b]);
    }
  }
};

using Stager = StagerT<cd>;

struct TreeInfo {
  int64_t n = 0;
  int32_t nc = 0;
  std::vector<int32_t> leaves;              // leaf cluster ids, by position
  std::vector<int32_t> leaf_first, leaf_cnt;  // per cluster: its leaves in `leaves`
  std::vector<std::vector<int32_t>> anc;    // per leaf: ancestors, root first, leaf last
};

int check_tree(int64_t n, const int64_t* perm, int32_t nc, const int64_t* off, const int64_t* size,
               const int32_t* parent, TreeInfo& T);

struct Timer {
  const char* name;
  double total_ms = 0.0;
  int64_t launches = 0;
};

struct PendingEvent {
  hipEvent_t a, b;
  int kernel;
};

struct LowpOp;  // low-precision (MFMA) operator state, defined with its kernels
void lowp_delete(LowpOp* lp);

}  // namespace uhm_detail

struct uhm_op {
  using cd = uhm_detail::cd;
  template <class T>
  using DevArray = uhm_detail::DevArray<T>;
  using CoupTile = uhm_detail::CoupTile;
  using Timer = uhm_detail::Timer;
  using PendingEvent = uhm_detail::PendingEvent;
  int kind = 0;  // 0 UH, 1 H
  int storage = UHM_C128;
  int64_t n = 0;
  int32_t nleaves = 0;
  uhm_op_info info{};

  DevArray<int32_t> perm, leaf_pos, leaf_n;
  DevArray<int32_t> iperm;  // user index -> cluster position
  // forward panels and partial sums
  DevArray<cd> F;
  DevArray<int64_t> fwd_off, poff;
  DevArray<int32_t> fwd_cols;
  DevArray<int2> ftiles;  // (leaf, tile) of every 64-column tile of the forward panels
  int32_t nftiles = 0;
  int64_t p_len = 0;
  // segments of the rank-space vector (u_sigma per cluster, or Y_b^* v per block)
  DevArray<int32_t> out_seg, seg_leaf0, seg_nleaf, seg_col;
  DevArray<int64_t> seg_start;
  int64_t nxh = 0;
  // couplings
  DevArray<cd> S;
  DevArray<CoupTile> ctiles;
  DevArray<int2> cblk;
  DevArray<int32_t> yh_grp, grp_t0, grp_nt;
  DevArray<int64_t> grp_start;
  int32_t nctiles = 0;
  int64_t nyh = 0;
  // factored couplings: first step t_b = S_{Y,b}^* u_sigma into the source vector after u
  DevArray<cd> FY;
  DevArray<uhm_detail::FacTile> factiles;
  int32_t nfactiles = 0;
  int64_t nsrc = 0;  // length of the coupling source vector (u, then the t_b)
  // backward panels
  DevArray<cd> B;
  DevArray<int64_t> bwd_off, zoff;
  DevArray<int32_t> bwd_cols, zmap;
  // streaming low-precision forms: F, S and B converted to the storage element
  DevArray<unsigned char> Fs, Ss, Bs;
  // symmetric storage (Remark 4.4): stored blocks applied as S_b and S_b^T, dense blocks
  // as A|_b and A|_b^T; the transposed products go through partial buffers
  bool sym = false;
  DevArray<uhm_detail::SymTile> stiles;
  DevArray<int32_t> csrc, grp_s0, grp_ns, bwd_tcol, fin_off, fin_cnt;
  DevArray<int64_t> tsrc, td_off, fsrc;
  int64_t ttot = 0, tdtot = 0;
  // workspace
  DevArray<cd> ws_p, ws_xh, ws_part, ws_yh, ws_tpart, ws_td;
  // timing
  bool timing = false;
  std::vector<Timer> timers;
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> free_events;

  uhm_detail::LowpOp* lp = nullptr;
  // staging of batched solve products (uhm_krylov_step)
  DevArray<unsigned char> stage_in, stage_out;
  int64_t stage_bytes = 0;

  ~uhm_op() {
    if (lp) uhm_detail::lowp_delete(lp);
    for (auto& e : pending) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    for (auto e : free_events) (void)hipEventDestroy(e);
  }
};

namespace uhm_detail {

enum {
  K_FORWARD = 0, K_REDUCE_FWD, K_COUPLING, K_REDUCE_COUP, K_BACKWARD,
  K_LP_GATHER, K_LP_FORWARD, K_LP_REDUCE_FWD, K_LP_COUPLING, K_LP_REDUCE_COUP, K_LP_BACKWARD, K_LP_SCATTER,
  K_SYM_COUPLING, K_SYM_REDUCE, K_SYM_BACKWARD, K_SYM_FINISH, K_FACTOR_IN, K_LP_FACTOR_IN,
  K_COUNT
};
extern const char* const kKernelNames[K_COUNT];

hipEvent_t get_event(uhm_op* op);

struct ScopedTiming {
  uhm_op* op;
  hipStream_t s;
  int k;
  hipEvent_t a = nullptr;
  ScopedTiming(uhm_op* o, hipStream_t st, int kernel) : op(o), s(st), k(kernel) {
    if (op->timing) {
      a = get_event(op);
      if (a) (void)hipEventRecord(a, s);
    }
  }
  ~ScopedTiming() {
    if (!a) return;
    hipEvent_t b = get_event(op);
    if (!b) return;
    (void)hipEventRecord(b, s);
    op->pending.push_back({a, b, k});
  }
};

inline bool in_bounds(int64_t off, int64_t count, int64_t len) { return off >= 0 && count >= 0 && off + count <= len; }

// Streaming low-precision forms (the complex128 layout with compact elements).
inline bool is_stream(int storage) { return storage == UHM_C64_STREAM || storage == UHM_BF16PAIR_STREAM; }
int stream_compact(uhm_op* op, hipStream_t s);
int stream_matvec(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, hipStream_t s);
int grow_workspace_fp64(uhm_op* op);

// Storage forms whose vectors and arithmetic are complex128.
inline bool is_c128(int storage) {
  return storage == UHM_C128 || storage == UHM_C128_MULTI || storage == UHM_C128_SYM || storage == UHM_C128_FACTORED ||
         storage == UHM_C128_MULTI_FACTORED;
}

int common_tree_upload(uhm_op* op, const TreeInfo& T, const int64_t* perm, const int64_t* off, const int64_t* size,
                       hipStream_t s);

struct LowpBatch;
int lowp_batch_create(uhm_op* const* ops, int32_t nops, const void* const* X, const int64_t* ldx, void* const* Y,
                      const int64_t* ldy, const int32_t* nrhs, hipStream_t s, LowpBatch** out);
int lowp_batch_run(LowpBatch* b, hipStream_t s);
int lowp_batch_capture(LowpBatch* b, hipStream_t s);
int lowp_batch_tune(LowpBatch* b, hipStream_t s, int32_t* width_out, int32_t* order_out, double* ms_out);
void lowp_batch_delete(LowpBatch* b);

// Many-RHS storage forms (complex64, bf16 pairs, complex128): MFMA kernels, own device layout.
int lowp_upload(const uhm_host_operator* h, uhm_storage storage, hipStream_t s, const TreeInfo& T, uhm_op* op);
int lowp_matvec(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs, hipStream_t s);
// Products Y_k = A_k X_k of several distinct operators of one many-RHS storage form in
// shared stage launches.  Columns are complex128 vectors in user order, given per operator
// as device arrays of ncols[k] (1..64) pointers xcol[k], ycol[k].  Calls must not overlap
// (shared staging).
int lowp_step_products(uhm_op* const* ops, const cd* const* const* xcol, cd* const* const* ycol, const int32_t* ncols,
                       int32_t nops, hipStream_t s);

}  // namespace uhm_detail
