// DMRG engine of libmdmrg (host orchestration of device work).
#pragma once
#include <array>
#include <set>

#include "internal.h"
#include "model.h"

namespace mdmrg {

// ------------------------------------------------------------- op keys
// Symbolic identity of a block operator: kind + list of elementary
// operators (index order).  K_H: block Hamiltonian; K_N: normal product of
// the listed operators (all inside the block); K_C: stored complementary
// operator whose listed operators lie outside the block; K_X: complementary
// operator formed on the fly from normal operators at one step.
// K_Z: a linear combination of normal operators of the left block that
// replaces a set of N^L x C^R products by a smaller set (key = K_Z | n << 4 |
// id << 8, n = length of the combined normal operators)
enum Kind : int { K_H = 0, K_N = 1, K_C = 2, K_X = 3, K_Z = 4, K_I = 15 };
uint64_t make_key(int kind, const int *e, int n);
inline uint64_t ident_key() { return uint64_t(K_I); }

// ------------------------------------------------------------- MPS
struct SiteTensor {
  std::vector<int32_t> bl, bs, br;
  std::vector<int64_t> off;
  std::unordered_map<int64_t, int> idx;
  double *data = nullptr;
  int64_t size = 0;
  static int64_t key(int l, int s, int r) { return (int64_t(l) * 64 + s) * (int64_t(1) << 24) + r; }
  int find(int l, int s, int r) const {
    auto it = idx.find(key(l, s, r));
    return it == idx.end() ? -1 : it->second;
  }
  void add(int l, int s, int r, int64_t sz) {
    idx[key(l, s, r)] = int(bl.size());
    bl.push_back(l);
    bs.push_back(s);
    br.push_back(r);
    off.push_back(size);
    size += sz;
  }
};

// ------------------------------------------------------------- block ops
struct Group {
  QN delta;
  std::vector<int32_t> row, col;
  std::vector<int64_t> poff;
  std::vector<int32_t> pair_of_col;
  int64_t size = 0;
  int32_t n_ops = 0;
  int64_t base = 0;
};

struct OpSet {
  const Bond *bond = nullptr;
  std::vector<Group> groups;
  std::unordered_map<int64_t, int> gidx;
  std::unordered_map<uint64_t, std::pair<int, int>> ops;
  std::vector<uint64_t> order;
  double *arena = nullptr;
  int64_t arena_size = 0;
  bool laid_out = false;
  void add(uint64_t key, QN delta);
  void layout(Device *dev);
  void release(Device *dev);
  bool has(uint64_t key) const { return ops.count(key) != 0; }
  int group_of(uint64_t key) const { return ops.at(key).first; }
  // offset in arena of the block of op `key` acting on column sector c; -1 if none
  int64_t block(uint64_t key, int c, int *row = nullptr) const;
  ~OpSet() = default;
};

// reference to an operator used in a product: identity, stored, or combo
struct OpRef {
  int src = 0;  // 0 identity, 1 stored (env), 2 combo
  uint64_t key = 0;
  bool operator<(const OpRef &o) const { return src != o.src ? src < o.src : key < o.key; }
  bool operator==(const OpRef &o) const { return src == o.src && key == o.key; }
};

// ------------------------------------------------------------- pair tasks
struct Ref {
  int slot = 0;
  int64_t off = 0;
  int ld = 0;
};
struct PairTask {
  int32_t out;  // index into output block table
  Ref A, X, B;
  bool tA = false, idA = false, tB = false, idB = false;
  int m, k1, k2, n;  // op(A): m x k1, X: k1 x k2, op(B): k2 x n
  double alpha;
};
struct OutBlk {
  int slot;
  int64_t off;
  int m, n, ld;
};
struct Chunk {
  DevPlan *p1 = nullptr, *p2 = nullptr;
  // split-K: phase 2 wrote n_split partial copies (slot 7, stride = output
  // buffer length); reduce them, in a fixed order, into these blocks
  DevReduce *red = nullptr;
};
struct TwoPhasePlan {
  std::vector<Chunk> chunks;
  int64_t scratch = 0;  // doubles
  double flop = 0.0;
  double bytes = 0.0;  // algorithmic HBM bytes: operands once, outputs once, intermediates twice
  int64_t n_gemm = 0;
  int n_split = 1;
  // algorithmic FLOP by the smaller output side min(m, n) of each GEMM,
  // bins [1,16) [16,32) [32,48) [48,64) [64,128) [128,256) [256,512) [512,inf)
  static constexpr int kHistBins = 8;
  double hist_flop[kHistBins] = {};
  void hist_add(int m, int n, double f) {
    static const int edges[kHistBins - 1] = {16, 32, 48, 64, 128, 256, 512};
    const int s = m < n ? m : n;
    int b = 0;
    while (b < kHistBins - 1 && s >= edges[b]) ++b;
    hist_flop[b] += f;
  }
  void release(Device *d) {
    for (auto &c : chunks) {
      dev_plan_free(d, c.p1);
      dev_plan_free(d, c.p2);
      dev_reduce_free(d, c.red);
    }
    chunks.clear();
    scratch = 0;
    flop = 0.0;
    bytes = 0.0;
    n_gemm = 0;
    n_split = 1;
    for (double &h : hist_flop) h = 0.0;
  }
};

// ------------------------------------------------------------- psi layout
struct PsiBlk {
  int a, s1, s2, b, m, n;
  int64_t off;
};
struct PsiLayout {
  std::vector<PsiBlk> blk;
  std::unordered_map<int64_t, int> idx;  // (a,s1,s2,b) -> block
  int64_t n_elem = 0;
  static int64_t key(int a, int s1, int s2, int b) {
    return ((int64_t(a) * 16 + s1) * 16 + s2) * (int64_t(1) << 24) + b;
  }
  int find(int a, int s1, int s2, int b) const {
    auto it = idx.find(key(a, s1, s2, b));
    return it == idx.end() ? -1 : it->second;
  }
};

struct Stats {
  double t_diag_h = 0, t_ren = 0, t_tables = 0, t_diag_d = 0, t_stvec = 0, t_other = 0;
  double heff_flop = 0, n_matvec = 0;
  double heff_flop_split = 0, n_matvec_split = 0;
};

// ------------------------------------------------------------- context
struct Context {
  Device *dev = nullptr;
  std::string err;
  Hamiltonian ham;
  bool have_ham = false;
  std::vector<Bond> bonds;
  std::vector<SiteTensor> A;
  bool have_mps = false;
  std::vector<std::unique_ptr<OpSet>> Lenv, Renv;  // by bond
  // current bond
  int cur = -1;
  PsiLayout psi;
  std::unique_ptr<OpSet> Lx, Rx;  // combos of this bond
  TwoPhasePlan heff;
  DevDiag *diag = nullptr;
  double *T_scratch = nullptr;
  int64_t T_scratch_n = 0;
  double *P_scratch = nullptr;  // split-K partial outputs
  int64_t P_scratch_n = 0;
  int64_t heff_terms = 0;
  Stats stats;
  int64_t scratch_limit = int64_t(1) << 30;  // doubles of phase-1 scratch (8 GB)
  // doubles of on-the-fly combinations formed at once by a renormalisation
  // (the new block's operators are renormalised in batches that fit)
  int64_t ren_combo_limit = int64_t(1) << 28;
  // Ritz vectors kept at a thick restart of the Davidson subspace
  // (MDMRG_OPT_DAVIDSON_KEEP)
  int davidson_keep = 2;
  bool davidson_olsen = false;  // Olsen correction vector (MDMRG_OPT_DAVIDSON_OLSEN)
  int floor_checks = 0;  // FP64 floor-check products of the last split Davidson
  int mixed_handover = 1;  // Ritz vectors handed from one mixed stage to the next
  // 3xBF16 mixed solves pass through an FP32 stage (MDMRG_OPT_MIXED_LADDER)
  bool mixed_ladder = false;
  // a mixed solve whose split stage stops above the FP64 tolerance continues
  // with split stages on the defect-corrected operator (MDMRG_OPT_MIXED_CORRECT)
  bool mixed_correct = false;
  // defect correction of the split products of davidson(): w += C v with
  // C = d x0^T + x0 d^T - gamma x0 x0^T, gamma = x0.d; corr = [x0 | d]
  const double *corr = nullptr;
  double corr_gamma = 0.0;
  void davidson_product(const double *v, double *w, int prec);
  int keep_envs = 1;  // blocks kept per bond (MDMRG_OPT_KEEP_ENVS): 1 all, 0/2/3 see prepare()
  bool compress = true;    // interpolative compression of the N^L x C^R products
  // graph replay of the H_eff product (MDMRG_OPT_GRAPH): captured per bond and
  // precision once the first products have tuned the kernel variants
  bool use_graph = false;
  DevGraph *graph64 = nullptr, *graph32 = nullptr, *graphbf3 = nullptr, *graphbf6 = nullptr;
  double *xg = nullptr, *yg = nullptr;  // FP64 staging of x and y for the graph
  int64_t xg_n = 0;
  int eager64 = 0, eager32 = 0, eagerbf3 = 0, eagerbf6 = 0;  // eager products at the current bond
  void set_graph(bool on);
  void release_graphs();

  ~Context();
  void reset_envs();
  void release_bond();
  // steps
  std::unique_ptr<OpSet> env_boundary(bool left, int bond);
  std::unique_ptr<OpSet> renorm_left(const OpSet &L, int site);   // L(bond site) -> L(bond site+1)
  std::unique_ptr<OpSet> renorm_right(const OpSet &R, int site);  // R(bond site+1) -> R(bond site)
  void prepare(int l);
  void build_heff(int l);
  void heff_apply(const double *x, double *y, int prec = 0);
  void heff_diag(double *d);
  // prec: matrix-vector precision (0 FP64, 1 FP32, 2 3xBF16, 3 6xBF16); stall_floor
  // >= 0: stop when the residual stops decreasing (split-precision phase):
  // no 10% gain over 4 products within twice stall_floor (the measured
  // noise floor of the split operator), over 24 within 20 times it, over 64
  // elsewhere
  // V0 (k0 vectors, the first equal to x): further start vectors; Vout
  // (kout vectors): receives the lowest Ritz vectors of the final subspace,
  // their number in *k_written
  int davidson(double *x, double tol, int max_iter, int m_max, double *energy, double *resid, int *n_mv,
               int prec = 0, double stall_floor = -1.0, const double *V0 = nullptr, int k0 = 0,
               double *Vout = nullptr, int kout = 0, int *k_written = nullptr,
               const double *hx_start = nullptr);
  // split-precision Davidson to tol_split, then FP64 Davidson to tol
  int davidson_mixed(double *x, double tol, int prec_split, double tol_split, int max_iter, int m_max,
                     double *energy, double *resid, int *n_mv64, int *n_mv_split);
  // FP32 shadows of the current bond's operators and vectors
  float *L32 = nullptr, *R32 = nullptr, *Lx32 = nullptr, *Rx32 = nullptr, *x32 = nullptr, *y32 = nullptr;
  void ensure_fp32();
  void decimate(const double *x, int D, int dir, double *trunc, double *svn, double *shalf);
  void stvec(const double *x_old, int l_old, int dir, const PsiLayout &old_layout, double *x_new,
             const PsiLayout &new_layout);
  // after decimate(dir): environment of the grown block, then bond l+dir;
  // prec 0 FP64, 1 FP32, 2 3xBF16, 3 6xBF16 products for that block's GEMMs (the
  // operators are stored as FP64 either way)
  void renormalize(int dir, int prec = 0);
  int ren_prec = 0;  // precision form of the renormalisation GEMMs in progress
  int last_decimated = 0;  // direction of the last decimation at the current bond (0 = none)
  int prev_l = -1, prev_dir = 0;
  PsiLayout prev_psi;
  PsiLayout make_layout(int l) const;
  // 0, or -5 (ENOCONV) when a Davidson solve of the sweep missed tol
  int sweep(int n_sweeps, const int *D, int n_sched, double tol, double *energies);
  void ensure_scratch(int64_t n);
  void run_plan(const TwoPhasePlan &p, Bases &b, int tag = 0, int prec = 0);
};

}  // namespace mdmrg
