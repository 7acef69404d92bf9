// Internal declarations of libmdmrg: quantum numbers, block-sparse storage,
// the grouped-GEMM task format and the device layer (implemented in
// device.hip with HIP kernels and rocSOLVER).
#pragma once

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

namespace mdmrg {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};
#define MDMRG_REQUIRE(cond, code, msg)                                     \
  do {                                                                     \
    if (!(cond)) throw ::mdmrg::Error((code), (msg));                      \
  } while (0)

// --------------------------------------------------------- quantum numbers
// (N, 0) for spinless fermions, (N_up, N_down) for spin-1/2 fermions.
struct QN {
  int a = 0, b = 0;
  QN() = default;
  QN(int a_, int b_) : a(a_), b(b_) {}
  QN operator+(const QN &o) const { return QN(a + o.a, b + o.b); }
  QN operator-(const QN &o) const { return QN(a - o.a, b - o.b); }
  bool operator==(const QN &o) const { return a == o.a && b == o.b; }
  bool operator!=(const QN &o) const { return !(*this == o); }
  bool operator<(const QN &o) const { return a != o.a ? a < o.a : b < o.b; }
  int parity() const { return (a + b) & 1; }
  int64_t key() const { return (int64_t(a) + 4096) * 8192 + (b + 4096); }
};

// A bond: sorted list of sectors.
struct Bond {
  std::vector<QN> qn;
  std::vector<int> dim;
  std::unordered_map<int64_t, int> index;
  int find(const QN &q) const {
    auto it = index.find(q.key());
    return it == index.end() ? -1 : it->second;
  }
  void rebuild_index() {
    index.clear();
    for (size_t i = 0; i < qn.size(); ++i) index[qn[i].key()] = int(i);
  }
  int total() const {
    int t = 0;
    for (int d : dim) t += d;
    return t;
  }
};

// ------------------------------------------------------ grouped GEMM tasks
// C(m x n) (+)= sum_seg alpha * op(A)(m x k) * op(B)(k x n), row-major,
// every pointer given as (slot, element offset).  One workgroup owns one
// output tile, so accumulation is deterministic and atomic-free.
enum : uint8_t { SEG_TA = 1, SEG_TB = 2, SEG_AID = 4 };
struct GSeg {
  int64_t a_off, b_off;
  double alpha;
  int32_t k, lda, ldb;
  uint8_t a_slot, b_slot, flags, pad;
};
struct GOut {
  int64_t c_off;
  int32_t m, n, ldc;
  int32_t seg_begin, seg_count;
  uint8_t c_slot, accumulate, pad0, pad1;
};
struct GTile {
  int32_t out;
  int32_t ti, tj;  // tile row / column within the output (a tall a3 output has millions of tile rows)
};
constexpr int kSlots = 8;
struct Bases {
  double *p[kSlots];
};

struct GemmPlan {  // host side
  std::vector<GSeg> segs;
  std::vector<GOut> outs;
  double flop = 0.0;  // algorithmic 2mnk, identity segments excluded
  void clear() {
    segs.clear();
    outs.clear();
    flop = 0.0;
  }
};

// Diagonal outer-product task: D[i][j] += alpha * Ld[i*ls] * Rd[j*rs]
struct DiagTask {
  int64_t d_off, l_off, r_off;  // d in slot 0, l/r in their slots
  double alpha;
  int32_t m, n, ls, rs;
  uint8_t l_slot, r_slot, l_id, r_id;  // *_id: operator is identity
};

// -------------------------------------------------------------- device layer
struct Device;
// stream: the caller's HIP stream (not owned), or nullptr for a stream of
// the context's own
Device *dev_create(int device, void *stream);
void dev_destroy(Device *);
void *dev_alloc(Device *, size_t bytes);  // throws Error(ENOMEM)
void dev_free(Device *, void *);
void dev_h2d(Device *, void *dst, const void *src, size_t bytes);
void dev_d2h(Device *, void *dst, const void *src, size_t bytes);
void dev_d2d(Device *, void *dst, const void *src, size_t bytes);
void dev_zero(Device *, void *dst, size_t bytes);
void dev_sync(Device *);
size_t dev_free_bytes(Device *);
// Allocation budget of the device context: dev_alloc throws ENOMEM when the
// live bytes of the context would exceed it.  Default (and upper limit):
// 95% of the device memory free at creation; 0 restores the default.
void dev_set_budget(Device *, size_t bytes);
size_t dev_live_bytes(Device *);

// Tile variants of the grouped kernel: 64x64 output tiles (one tile list)
// split over waves as 0 k_gemm (2x4 waves), 1 k_gemm_w16 (4x4), 2 k_gemm_w4
// (2x2); 3 k_gemm_t128, 128x128 tiles (their own tile list) over 2x4 waves.
constexpr int kGemmVariants = 4;
// Precision forms of the grouped kernel: 0 FP64; 1 FP32 (FP32 operands,
// MFMA accumulation and results); 2 3xBF16 (FP32 operands and results, each
// product formed from BF16 hi / lo parts with FP32 accumulation); 3 6xBF16
// (the same with hi / mid / lo parts and six BF16 products).
constexpr int kPrecs = 4;

// Uploaded grouped-GEMM plan: 64x64 output tiles in launch order (outputs
// largest first, dealt to per-XCD queues; empty tiles pad the queues).
struct DevPlan {
  GSeg *segs = nullptr;
  GOut *outs = nullptr;
  GTile *tiles = nullptr, *tiles128 = nullptr;  // 64x64 and 128x128 tile lists
  int64_t n_tiles = 0, n_tiles128 = 0, n_outs = 0, n_segs = 0;
  double flop = 0.0;  // algorithmic FLOP of one launch
  // autotuner state per precision form: the first launches time one
  // variant each, then the fastest is kept (variant >= 0)
  int variant[kPrecs] = {-1, -1, -1, -1}, trials[kPrecs] = {0, 0, 0, 0};
  void *trial_ev[kPrecs][2 * kGemmVariants] = {};
  float trial_ms[kPrecs][kGemmVariants] = {};
};
DevPlan *dev_plan_upload(Device *, const GemmPlan &);
// v in 0..kGemmVariants-1: every later grouped launch of the device uses tile
// variant v (no autotuning); -1: autotune per plan (default)
void dev_force_variant(Device *, int v);
void dev_plan_free(Device *, DevPlan *);
// Bytes of the static per-device staging array of dev_gemm_run_noalloc.
constexpr size_t kNoAllocStagingBytes = size_t(16) << 20;
// FP64 grouped GEMM without any allocation: the plan goes into the static
// staging array of the device, the launch uses the forced variant or
// k_gemm_w4 and is waited for.  EINVAL (-1) if the plan does not fit.
void dev_gemm_run_noalloc(Device *, const GemmPlan &, const Bases &);
// prec 0: FP64 operands and results; prec 1 (FP32), 2 (3xBF16) and 3
// (6xBF16): FP32 operands and results (base pointers then address float
// arrays with the same element offsets)
void dev_gemm_run(Device *, DevPlan *, const Bases &, int tag = 0, int prec = 0);
void dev_d2f(Device *, const double *x, float *y, int64_t n);
void dev_f2d(Device *, const float *x, double *y, int64_t n);
// HIP-event timing of tagged grouped-GEMM launches (tag 1..6; untagged
// launches count as 6) and of graph replays (tags 7 FP64, 8 FP32, 9
// 3xBF16, 10 6xBF16): elapsed milliseconds, launch count and algorithmic
// FLOP since creation.
constexpr int kTags = 11;
void dev_timing_enable(Device *, bool on);
void dev_timing_collect(Device *, double ms[kTags], double launches[kTags], double flop[kTags]);
// Process-wide totals of the grouped kernel per precision form and tile
// variant over every context of the process since load (destroyed ones
// included).
void dev_timing_process(Device *, double ms[kPrecs][kGemmVariants], double launches[kPrecs][kGemmVariants],
                        double flop[kPrecs][kGemmVariants]);
// Stream capture of the context stream into a graph (no timing events and
// no host synchronisation inside), replay, and release.  A replay is timed
// as a whole under `tag` when timing is on.
struct DevGraph;
void dev_capture_begin(Device *);
DevGraph *dev_capture_end(Device *);
void dev_capture_abort(Device *);
void dev_graph_launch(Device *, DevGraph *, int tag, double flop);
void dev_graph_free(Device *, DevGraph *);

// Deterministic split-K reduction: y[off+i] += sum_{s<S} P[s*stride + off+i]
// over a list of blocks (off, len), s ascending.
struct DevReduce {
  int64_t *off = nullptr;
  int32_t *len = nullptr;
  int64_t n_blk = 0;
  int64_t max_len = 0;
  int n_split = 1;
  int64_t stride = 0;
};
DevReduce *dev_reduce_upload(Device *, const std::vector<int64_t> &off, const std::vector<int32_t> &len,
                             int n_split, int64_t stride);
void dev_reduce_free(Device *, DevReduce *);
void dev_reduce_run(Device *, const DevReduce *, const double *P, double *y, int prec);

struct DevDiag {
  DiagTask *tasks = nullptr;
  int32_t *blk_begin = nullptr;  // CSR over output blocks
  int64_t n_tasks = 0, n_blk = 0;
  int64_t *blk_off = nullptr;
  int32_t *blk_m = nullptr, *blk_n = nullptr;
};
DevDiag *dev_diag_upload(Device *, const std::vector<DiagTask> &, const std::vector<int64_t> &blk_off,
                         const std::vector<int32_t> &blk_m, const std::vector<int32_t> &blk_n);
void dev_diag_free(Device *, DevDiag *);
void dev_diag_run(Device *, const DevDiag *, const Bases &, double *d);

// FP64 vector primitives (deterministic reductions)
// out[i] = sum_k V[i*ldv + k] * x[k], i < m      (result on host)
void dev_multidot(Device *, const double *V, int64_t ldv, int m, const double *x, int64_t n, double *out_host);
// y[k] = beta*y[k] + sum_i c[i] * V[i*ldv + k]
void dev_lincomb(Device *, const double *V, int64_t ldv, int m, const double *c_host, double beta, double *y,
                 int64_t n);
void dev_axpy(Device *, double a, const double *x, double *y, int64_t n);
void dev_scale(Device *, double a, double *x, int64_t n);
// t[k] = r[k] / clamp(theta - d[k])  with |theta - d| >= eps
void dev_precond(Device *, const double *r, const double *d, double theta, double eps, double *t, int64_t n);
// Gaussian N(0,1) fill from a counter-based generator (splitmix64 + Box-Muller)
void dev_randn(Device *, double *x, int64_t n, uint64_t seed);
// Symmetric eigensolver (rocSOLVER dsyevd): A (n x n, overwritten by the
// eigenvectors, column k = eigenvector k), w ascending.  Device pointers.
void dev_syevd(Device *, double *A, int n, double *w);
// Gather: out[b][i*ncol + j] = E[col[j]*ldE + row0 + i] for a list of blocks
struct GatherBlk {
  int64_t out_off, e_off;  // out block, start of eigenvector storage
  int32_t rows, ncol, ldE, row0;
  int32_t col_begin;  // into the column index array
};
void dev_gather(Device *, const std::vector<GatherBlk> &, const std::vector<int32_t> &cols, const double *E,
                double *out, bool transpose_out);

// -------------------------------------------------------------- timing
double wall_seconds();

}  // namespace mdmrg
