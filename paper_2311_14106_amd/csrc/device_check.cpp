// Range-checking device layer: a host-only stand-in for device.hip, linked
// into libmdmrg_check.so instead of it (paper_2311_14106_amd.build,
// check=True).  It performs no arithmetic.  Device allocations get fake,
// never-reused addresses (nothing is backed by memory), and every access a
// kernel of the real layer would make -- each grouped-GEMM operand and output
// block, split-K partials and reductions, diagonal tasks, gathers, vector
// operations, copies -- is checked against the live allocations on the host;
// an access outside them throws EDEVICE naming the launch and the range.
// The live and peak allocated bytes are exported, so the planner's index
// arithmetic and the memory footprint of a workload can be checked on the
// CPU at sizes no test GPU run covers.
//
// Host reads of device data see synthetic values: dot products read 1, and
// the eigenvalues of every per-sector eigenproblem are exp(-8 (n-1-j)/n),
// j = 0..n-1 ascending, so a truncation keeps the same fraction of every
// sector (kept dimensions proportional to the sector dimensions).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>

#include "internal.h"

namespace mdmrg {

struct Device {
  int id = 0;
  std::map<uint64_t, size_t> live;  // fake base address -> bytes
  size_t live_bytes = 0, peak_bytes = 0, budget_bytes = 0, budget_default = 0;
  uint64_t next = uint64_t(1) << 44;
  std::map<uint64_t, int> eig;  // eigenvalue arrays written by dev_syevd: address -> n
  int force_variant = -1;
  int64_t checked_launches = 0;
  double flop = 0.0;  // algorithmic FLOP of every grouped launch checked
  size_t trace_bytes = 0;  // MDMRG_CHECK_TRACE_GB: print allocations and frees of at least this size
};

static std::mutex g_mu;
static Device *g_last = nullptr;  // the most recently created device layer

static void check_range(Device *d, const void *p, uint64_t bytes, const char *what) {
  if (bytes == 0) return;
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  auto it = d->live.upper_bound(a);
  if (it == d->live.begin())
    throw Error(-3, std::string("range check: ") + what + " at an address below every allocation");
  --it;
  if (a < it->first || a + bytes > it->first + it->second)
    throw Error(-3, std::string("range check: ") + what + " [" + std::to_string(a - it->first) + ", " +
                        std::to_string(a - it->first + bytes) + ") outside its allocation of " +
                        std::to_string(it->second) + " bytes");
}

Device *dev_create(int device, void *) {
  auto *d = new Device();
  d->id = device;
  d->budget_bytes = d->budget_default = size_t(1) << 50;
  if (const char *t = getenv("MDMRG_CHECK_TRACE_GB")) d->trace_bytes = size_t(atof(t) * 1e9);
  std::lock_guard<std::mutex> lk(g_mu);
  g_last = d;
  return d;
}
void dev_destroy(Device *d) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_last == d) g_last = nullptr;
  delete d;
}
void *dev_alloc(Device *d, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (d->live_bytes + bytes > d->budget_bytes)
    throw Error(-2, "device memory budget exceeded: " + std::to_string(bytes) + " bytes requested, " +
                        std::to_string(d->live_bytes) + " in use of " + std::to_string(d->budget_bytes));
  const uint64_t a = d->next;
  d->next += (bytes + 4095 + 4096) & ~uint64_t(4095);  // a gap after every allocation
  d->live[a] = bytes;
  d->live_bytes += bytes;
  d->peak_bytes = std::max(d->peak_bytes, d->live_bytes);
  if (d->trace_bytes && bytes >= d->trace_bytes)
    fprintf(stderr, "[check] alloc %.2f GB -> live %.2f GB\n", bytes / 1e9, d->live_bytes / 1e9);
  return reinterpret_cast<void *>(a);
}
void dev_free(Device *d, void *p) {
  if (!p) return;
  auto it = d->live.find(reinterpret_cast<uint64_t>(p));
  MDMRG_REQUIRE(it != d->live.end(), -3, "range check: free of an address that is not a live allocation");
  d->live_bytes -= it->second;
  if (d->trace_bytes && it->second >= d->trace_bytes)
    fprintf(stderr, "[check] free %.2f GB -> live %.2f GB\n", it->second / 1e9, d->live_bytes / 1e9);
  d->eig.erase(it->first);
  d->live.erase(it);
}
void dev_set_budget(Device *d, size_t bytes) {
  d->budget_bytes = bytes ? std::min(bytes, d->budget_default) : d->budget_default;
}
size_t dev_live_bytes(Device *d) { return d->live_bytes; }
size_t dev_free_bytes(Device *d) { return d->budget_bytes - std::min(d->budget_bytes, d->live_bytes); }
void dev_h2d(Device *d, void *dst, const void *, size_t b) { check_range(d, dst, b, "host-to-device copy"); }
void dev_d2h(Device *d, void *dst, const void *src, size_t b) {
  check_range(d, src, b, "device-to-host copy");
  double *o = static_cast<double *>(dst);
  const uint64_t a = reinterpret_cast<uint64_t>(src);
  // synthetic eigenvalues where dev_syevd wrote them, else zeros
  std::memset(dst, 0, b);
  for (auto &e : d->eig) {
    const uint64_t lo = std::max(a, e.first), hi = std::min(a + b, e.first + 8 * uint64_t(e.second));
    for (uint64_t x = lo; x + 8 <= hi; x += 8) {
      const int n = e.second, j = int((x - e.first) / 8);
      o[(x - a) / 8] = std::exp(-8.0 * double(n - 1 - j) / double(n));
    }
  }
}
void dev_d2d(Device *d, void *dst, const void *src, size_t b) {
  check_range(d, dst, b, "device copy (destination)");
  check_range(d, src, b, "device copy (source)");
}
void dev_zero(Device *d, void *dst, size_t b) { check_range(d, dst, b, "zero fill"); }
void dev_sync(Device *) {}

DevPlan *dev_plan_upload(Device *, const GemmPlan &plan) {
  // the plan stays on the host: segs / outs point to host copies
  auto *dp = new DevPlan();
  dp->n_outs = int64_t(plan.outs.size());
  dp->n_segs = int64_t(plan.segs.size());
  dp->segs = new GSeg[std::max<size_t>(1, plan.segs.size())];
  dp->outs = new GOut[std::max<size_t>(1, plan.outs.size())];
  std::copy(plan.segs.begin(), plan.segs.end(), dp->segs);
  std::copy(plan.outs.begin(), plan.outs.end(), dp->outs);
  // the device kernels' 32-bit offset limits (plan_check of the HIP layer):
  // buffer-load byte offsets inside one 128 x 128 tile's K step of at most
  // 16, for 8-byte elements, below 2^30
  for (const GOut &o : plan.outs)
    for (int q = 0; q < o.seg_count; ++q) {
      const GSeg &g = plan.segs[o.seg_begin + q];
      const int64_t ta = (g.flags & SEG_TA) ? int64_t(16) * g.lda + 128 : int64_t(128) * g.lda + 16;
      const int64_t tb = (g.flags & SEG_TB) ? int64_t(128) * g.ldb + 16 : int64_t(16) * g.ldb + 128;
      MDMRG_REQUIRE(8 * ta < (int64_t(1) << 30) && 8 * tb < (int64_t(1) << 30), -6,
                    "grouped GEMM: leading dimension too large for 32-bit tile offsets");
    }
  for (const GOut &o : plan.outs) {
    dp->n_tiles += int64_t((o.m + 63) / 64) * ((o.n + 63) / 64);
    dp->n_tiles128 += int64_t((o.m + 127) / 128) * ((o.n + 127) / 128);
    for (int q = 0; q < o.seg_count; ++q) {
      const GSeg &g = plan.segs[o.seg_begin + q];
      if (!(g.flags & SEG_AID)) dp->flop += 2.0 * o.m * o.n * g.k;
    }
  }
  return dp;
}
void dev_force_variant(Device *d, int v) { d->force_variant = v; }
void dev_plan_free(Device *, DevPlan *p) {
  if (!p) return;
  delete[] p->segs;
  delete[] p->outs;
  delete p;
}

static void check_plan(Device *d, const GOut *outs, int64_t n_outs, const GSeg *segs, const Bases &b, int prec) {
  const uint64_t es = prec == 0 ? 8 : 4;
  for (int64_t i = 0; i < n_outs; ++i) {
    const GOut &o = outs[i];
    MDMRG_REQUIRE(o.m >= 1 && o.n >= 1 && o.ldc >= o.n, -3, "range check: bad output shape");
    check_range(d, reinterpret_cast<const char *>(b.p[o.c_slot]) + es * o.c_off,
                es * (uint64_t(o.m - 1) * o.ldc + o.n), "grouped GEMM output");
    for (int q = 0; q < o.seg_count; ++q) {
      const GSeg &g = segs[o.seg_begin + q];
      if (g.k == 0) continue;
      if (!(g.flags & SEG_AID)) {
        const uint64_t last = (g.flags & SEG_TA) ? uint64_t(g.k - 1) * g.lda + o.m : uint64_t(o.m - 1) * g.lda + g.k;
        check_range(d, reinterpret_cast<const char *>(b.p[g.a_slot]) + es * g.a_off, es * last,
                    "grouped GEMM A operand");
      } else {
        MDMRG_REQUIRE(g.k == o.m, -3, "range check: identity left factor with k != m");
      }
      const uint64_t lastb = (g.flags & SEG_TB) ? uint64_t(o.n - 1) * g.ldb + g.k : uint64_t(g.k - 1) * g.ldb + o.n;
      check_range(d, reinterpret_cast<const char *>(b.p[g.b_slot]) + es * g.b_off, es * lastb,
                  "grouped GEMM B operand");
    }
  }
  d->checked_launches += 1;
}
void dev_gemm_run(Device *d, DevPlan *p, const Bases &b, int, int prec) {
  if (!p || p->n_outs == 0) return;
  MDMRG_REQUIRE(prec >= 0 && prec < kPrecs, -6, "grouped GEMM: unknown precision form");
  check_plan(d, p->outs, p->n_outs, p->segs, b, prec);
  d->flop += p->flop;
}
void dev_gemm_run_noalloc(Device *d, const GemmPlan &plan, const Bases &b) {
  check_plan(d, plan.outs.data(), int64_t(plan.outs.size()), plan.segs.data(), b, 0);
}
void dev_d2f(Device *d, const double *x, float *y, int64_t n) {
  check_range(d, x, 8 * uint64_t(n), "FP64 to FP32 conversion (source)");
  check_range(d, y, 4 * uint64_t(n), "FP64 to FP32 conversion (destination)");
}
void dev_f2d(Device *d, const float *x, double *y, int64_t n) {
  check_range(d, x, 4 * uint64_t(n), "FP32 to FP64 conversion (source)");
  check_range(d, y, 8 * uint64_t(n), "FP32 to FP64 conversion (destination)");
}

void dev_timing_enable(Device *, bool) {}
void dev_timing_collect(Device *, double ms[kTags], double launches[kTags], double flop[kTags]) {
  for (int i = 0; i < kTags; ++i) ms[i] = launches[i] = flop[i] = 0.0;
}
void dev_timing_process(Device *, double ms[kPrecs][kGemmVariants], double launches[kPrecs][kGemmVariants],
                        double flop[kPrecs][kGemmVariants]) {
  for (int p = 0; p < kPrecs; ++p)
    for (int v = 0; v < kGemmVariants; ++v) ms[p][v] = launches[p][v] = flop[p][v] = 0.0;
}
struct DevGraph {
  int unused = 0;
};
void dev_capture_begin(Device *) {}
DevGraph *dev_capture_end(Device *) { return new DevGraph(); }
void dev_capture_abort(Device *) {}
void dev_graph_launch(Device *, DevGraph *, int, double) {}
void dev_graph_free(Device *, DevGraph *g) { delete g; }

DevReduce *dev_reduce_upload(Device *, const std::vector<int64_t> &off, const std::vector<int32_t> &len,
                             int n_split, int64_t stride) {
  // host copies of the block list
  auto *r = new DevReduce();
  r->n_blk = int64_t(off.size());
  r->n_split = n_split;
  r->stride = stride;
  r->off = new int64_t[std::max<size_t>(1, off.size())];
  r->len = new int32_t[std::max<size_t>(1, len.size())];
  std::copy(off.begin(), off.end(), r->off);
  std::copy(len.begin(), len.end(), r->len);
  for (int32_t l : len) r->max_len = std::max<int64_t>(r->max_len, l);
  return r;
}
void dev_reduce_free(Device *, DevReduce *r) {
  if (!r) return;
  delete[] r->off;
  delete[] r->len;
  delete r;
}
void dev_reduce_run(Device *d, const DevReduce *r, const double *P, double *y, int prec) {
  if (!r) return;
  const uint64_t es = prec == 0 ? 8 : 4;
  for (int64_t i = 0; i < r->n_blk; ++i) {
    check_range(d, reinterpret_cast<const char *>(y) + es * r->off[i], es * r->len[i], "split-K reduction output");
    for (int q = 0; q < r->n_split; ++q)
      check_range(d, reinterpret_cast<const char *>(P) + es * (q * r->stride + r->off[i]), es * r->len[i],
                  "split-K partial");
  }
}

DevDiag *dev_diag_upload(Device *, const std::vector<DiagTask> &tasks, const std::vector<int64_t> &blk_off,
                         const std::vector<int32_t> &blk_m, const std::vector<int32_t> &blk_n) {
  auto *dd = new DevDiag();
  dd->n_tasks = int64_t(tasks.size());
  dd->n_blk = int64_t(blk_off.size());
  dd->tasks = new DiagTask[std::max<size_t>(1, tasks.size())];
  std::copy(tasks.begin(), tasks.end(), dd->tasks);
  dd->blk_off = new int64_t[std::max<size_t>(1, blk_off.size())];
  dd->blk_m = new int32_t[std::max<size_t>(1, blk_m.size())];
  dd->blk_n = new int32_t[std::max<size_t>(1, blk_n.size())];
  std::copy(blk_off.begin(), blk_off.end(), dd->blk_off);
  std::copy(blk_m.begin(), blk_m.end(), dd->blk_m);
  std::copy(blk_n.begin(), blk_n.end(), dd->blk_n);
  return dd;
}
void dev_diag_free(Device *, DevDiag *p) {
  if (!p) return;
  delete[] p->tasks;
  delete[] p->blk_off;
  delete[] p->blk_m;
  delete[] p->blk_n;
  delete p;
}
void dev_diag_run(Device *d, const DevDiag *p, const Bases &b, double *out) {
  if (!p) return;
  std::unordered_map<int64_t, int64_t> blk;
  for (int64_t i = 0; i < p->n_blk; ++i) {
    check_range(d, out + p->blk_off[i], 8 * uint64_t(p->blk_m[i]) * p->blk_n[i], "diagonal output block");
    blk[p->blk_off[i]] = i;
  }
  for (int64_t t = 0; t < p->n_tasks; ++t) {
    const DiagTask &k = p->tasks[t];
    auto it = blk.find(k.d_off);
    MDMRG_REQUIRE(it != blk.end(), -3, "range check: diagonal task of an unknown output block");
    MDMRG_REQUIRE(k.m == p->blk_m[it->second] && k.n == p->blk_n[it->second], -3,
                  "range check: diagonal task shape differs from its block");
    if (!k.l_id) check_range(d, b.p[k.l_slot] + k.l_off, 8 * (uint64_t(k.m - 1) * k.ls + 1), "diagonal left operand");
    if (!k.r_id) check_range(d, b.p[k.r_slot] + k.r_off, 8 * (uint64_t(k.n - 1) * k.rs + 1), "diagonal right operand");
  }
}

void dev_multidot(Device *d, const double *V, int64_t ldv, int m, const double *x, int64_t n, double *out_host) {
  for (int i = 0; i < m; ++i) {
    check_range(d, V + i * ldv, 8 * uint64_t(n), "multi-dot row");
    out_host[i] = 1.0;
  }
  check_range(d, x, 8 * uint64_t(n), "multi-dot vector");
}
void dev_lincomb(Device *d, const double *V, int64_t ldv, int m, const double *, double, double *y, int64_t n) {
  for (int i = 0; i < m; ++i) check_range(d, V + i * ldv, 8 * uint64_t(n), "linear combination row");
  check_range(d, y, 8 * uint64_t(n), "linear combination output");
}
void dev_axpy(Device *d, double, const double *x, double *y, int64_t n) {
  check_range(d, x, 8 * uint64_t(n), "axpy x");
  check_range(d, y, 8 * uint64_t(n), "axpy y");
}
void dev_scale(Device *d, double, double *x, int64_t n) { check_range(d, x, 8 * uint64_t(n), "scale"); }
void dev_precond(Device *d, const double *r, const double *dg, double, double, double *t, int64_t n) {
  check_range(d, r, 8 * uint64_t(n), "preconditioner residual");
  check_range(d, dg, 8 * uint64_t(n), "preconditioner diagonal");
  check_range(d, t, 8 * uint64_t(n), "preconditioner output");
}
void dev_randn(Device *d, double *x, int64_t n, uint64_t) { check_range(d, x, 8 * uint64_t(n), "random fill"); }
void dev_syevd(Device *d, double *A, int n, double *w) {
  if (n <= 0) return;
  check_range(d, A, 8 * uint64_t(n) * n, "eigensolver matrix");
  check_range(d, w, 8 * uint64_t(n), "eigensolver values");
  d->eig[reinterpret_cast<uint64_t>(w)] = n;
}
void dev_gather(Device *d, const std::vector<GatherBlk> &blks, const std::vector<int32_t> &cols, const double *E,
                double *out, bool) {
  for (const GatherBlk &g : blks) {
    check_range(d, out + g.out_off, 8 * uint64_t(g.rows) * g.ncol, "gather output");
    for (int j = 0; j < g.ncol; ++j)
      check_range(d, E + g.e_off + int64_t(cols.at(g.col_begin + j)) * g.ldE + g.row0, 8 * uint64_t(g.rows),
                  "gather source column");
  }
}

double wall_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace mdmrg

// Exported only by the range-checking build: the allocation record of the
// most recently created context, and fake device buffers for its calls.
extern "C" {
int64_t mdmrg_check_live_bytes(void) {
  std::lock_guard<std::mutex> lk(mdmrg::g_mu);
  return mdmrg::g_last ? int64_t(mdmrg::g_last->live_bytes) : -1;
}
int64_t mdmrg_check_peak_bytes(void) {
  std::lock_guard<std::mutex> lk(mdmrg::g_mu);
  return mdmrg::g_last ? int64_t(mdmrg::g_last->peak_bytes) : -1;
}
void mdmrg_check_reset_peak(void) {
  std::lock_guard<std::mutex> lk(mdmrg::g_mu);
  if (mdmrg::g_last) mdmrg::g_last->peak_bytes = mdmrg::g_last->live_bytes;
}
double mdmrg_check_flop(void) {
  std::lock_guard<std::mutex> lk(mdmrg::g_mu);
  return mdmrg::g_last ? mdmrg::g_last->flop : -1.0;
}
int64_t mdmrg_check_launches(void) {
  std::lock_guard<std::mutex> lk(mdmrg::g_mu);
  return mdmrg::g_last ? mdmrg::g_last->checked_launches : -1;
}
void *mdmrg_check_alloc(int64_t bytes) {
  std::lock_guard<std::mutex> lk(mdmrg::g_mu);
  return mdmrg::g_last ? mdmrg::dev_alloc(mdmrg::g_last, size_t(bytes)) : nullptr;
}
}
