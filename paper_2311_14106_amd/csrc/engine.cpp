// DMRG engine: block operators, normal/complementary partition of Eq. (1)
// at every bond, renormalisation, the task lists of the effective
// Hamiltonian, Davidson, density-matrix decimation, start vectors, sweeps.
//
// Notation: a term of Eq. (1) is an index-ordered product of elementary
// operators.  At a bond the chain is split into the left block L (sites < l),
// the two explicit sites S1 = l, S2 = l+1 and the right block R (sites > l+1).
// Each term is written as (L part)(S1 part)(S2 part)(R part) and routed to
// exactly one product  X_L (x) O_S (x) X_R  of stored or on-the-fly block
// operators (normal operators on L, complementary operators on R, plus the
// few complementary operators of L that the sums need), so that the number
// of products is O(n^2) and every product is a pair of dense sector GEMMs.
#include <algorithm>
#include <atomic>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <numeric>
#include <unordered_map>
#include <unordered_set>

#include "engine.h"

namespace mdmrg {

// Device work vectors of one call, freed when the call returns or throws.
namespace {
struct DevVecs {
  Device *d;
  std::vector<void *> held;
  explicit DevVecs(Device *dev) : d(dev) {}
  double *get(int64_t n) {
    held.reserve(held.size() + 1);
    double *q = static_cast<double *>(dev_alloc(d, sizeof(double) * size_t(n)));
    held.push_back(q);
    return q;
  }
  void release(double *q) {  // free one vector before the scope ends
    for (size_t i = 0; i < held.size(); ++i)
      if (held[i] == q) {
        held.erase(held.begin() + i);
        dev_free(d, q);
        return;
      }
  }
  DevVecs(const DevVecs &) = delete;
  DevVecs &operator=(const DevVecs &) = delete;
  ~DevVecs() {
    for (void *q : held) {
      try {
        dev_free(d, q);
      } catch (...) {
      }
    }
  }
};
}  // namespace

uint64_t make_key(int kind, const int *e, int n) {
  uint64_t k = uint64_t(kind) | (uint64_t(n) << 4);
  for (int i = 0; i < n; ++i) k |= uint64_t(e[i] + 1) << (8 + 13 * i);
  return k;
}
static int key_kind(uint64_t k) { return int(k & 15); }
static int key_n(uint64_t k) { return int((k >> 4) & 15); }
static int key_parity(uint64_t k) {
  const int kd = key_kind(k);
  if (kd == K_H || kd == K_I) return 0;
  return key_n(k) & 1;
}
static int parity_of_state(int s) { return __builtin_popcount(unsigned(s)) & 1; }

// ------------------------------------------------------------------ OpSet
void OpSet::add(uint64_t key, QN delta) {
  if (ops.count(key)) return;
  auto it = gidx.find(delta.key());
  int g;
  if (it == gidx.end()) {
    g = int(groups.size());
    gidx[delta.key()] = g;
    groups.emplace_back();
    groups.back().delta = delta;
  } else {
    g = it->second;
  }
  ops[key] = {g, groups[g].n_ops++};
  order.push_back(key);
}

void OpSet::layout(Device *dev) {
  int64_t base = 0;
  const int nsec = int(bond->qn.size());
  for (auto &G : groups) {
    G.pair_of_col.assign(nsec, -1);
    G.row.clear();
    G.col.clear();
    G.poff.clear();
    G.size = 0;
    for (int c = 0; c < nsec; ++c) {
      const int r = bond->find(bond->qn[c] + G.delta);
      if (r < 0) continue;
      G.pair_of_col[c] = int(G.row.size());
      G.row.push_back(r);
      G.col.push_back(c);
      G.poff.push_back(G.size);
      G.size += int64_t(bond->dim[r]) * bond->dim[c];
    }
    G.base = base;
    base += (G.size * G.n_ops + 31) / 32 * 32;
  }
  arena_size = base;
  arena = (double *)dev_alloc(dev, sizeof(double) * std::max<int64_t>(1, arena_size));
  dev_zero(dev, arena, sizeof(double) * std::max<int64_t>(1, arena_size));
  laid_out = true;
}

void OpSet::release(Device *dev) {
  if (arena) dev_free(dev, arena);
  arena = nullptr;
}

int64_t OpSet::block(uint64_t key, int c, int *row) const {
  auto it = ops.find(key);
  if (it == ops.end()) return -1;
  const Group &G = groups[it->second.first];
  if (c < 0 || c >= int(G.pair_of_col.size())) return -1;
  const int p = G.pair_of_col[c];
  if (p < 0) return -1;
  if (row) *row = G.row[p];
  return G.base + int64_t(it->second.second) * G.size + G.poff[p];
}

// ------------------------------------------------------------------ helpers
struct Parts {
  int k[4] = {0, 0, 0, 0};
  int e[4][4];
};
// part 0: sites < s1, 1: site s1, 2: site s1+1, 3: sites > s1+1
static void split(const Hamiltonian &H, const Term &t, int s1, Parts &p) {
  for (int i = 0; i < t.n; ++i) {
    const int site = H.site_of(t.e[i]);
    const int part = site < s1 ? 0 : site == s1 ? 1 : site == s1 + 1 ? 2 : 3;
    p.e[part][p.k[part]++] = t.e[i];
  }
}
static QN q_sum(const Hamiltonian &H, const int *e, int n) {
  QN q;
  for (int i = 0; i < n; ++i) q = q + H.q_of_op(e[i]);
  return q;
}

// d x d site matrix list accumulated per (source operator)
struct SiteItem {
  std::vector<double> M;
  int parity = 0;
};

// ------------------------------------------------------------------ needs
static void need_left(const Hamiltonian &H, int bond, OpSet &S) {
  S.add(make_key(K_H, nullptr, 0), QN());
  for (int p = 0; p < H.ns * bond; ++p)
    for (int dag = 1; dag >= 0; --dag) {
      const int e = 2 * p + dag;
      S.add(make_key(K_N, &e, 1), H.q_of_op(e));
    }
  for (const Term &t : H.terms) {
    int in[4], out[4], ki = 0, ko = 0;
    for (int i = 0; i < t.n; ++i) {
      if (H.site_of(t.e[i]) < bond)
        in[ki++] = t.e[i];
      else
        out[ko++] = t.e[i];
    }
    if (ki == 2) S.add(make_key(K_N, in, 2), q_sum(H, in, 2));
    if (t.n == 4 && ki == 3) S.add(make_key(K_C, out, 1), QN() - q_sum(H, out, 1));
  }
}

static void need_right(const Hamiltonian &H, int bond, OpSet &S) {
  S.add(make_key(K_H, nullptr, 0), QN());
  for (int p = H.ns * bond; p < H.nso; ++p)
    for (int dag = 1; dag >= 0; --dag) {
      const int e = 2 * p + dag;
      S.add(make_key(K_N, &e, 1), QN() - H.q_of_op(e));
    }
  for (const Term &t : H.terms) {
    int out[4], ki = 0, ko = 0;
    for (int i = 0; i < t.n; ++i) {
      if (H.site_of(t.e[i]) >= bond)
        ++ki;
      else
        out[ko++] = t.e[i];
    }
    if (ki >= 1 && (ko == 1 || ko == 2)) S.add(make_key(K_C, out, ko), q_sum(H, out, ko));
  }
}

// content of on-the-fly complementary operators of a block: combo key ->
// list of (normal operator key, coefficient).  Left: terms with
// ext_L(t) = K and k_L >= 1, except the three-operator two-body part (kept
// as a stored operator).  Right: terms with ext_R(t) = K, k_R == 1 (|K|=3).
using Content = std::map<uint64_t, std::map<uint64_t, double>>;
static void combo_content(const Hamiltonian &H, bool left, int bond, const std::set<uint64_t> &wanted,
                          Content &out) {
  if (wanted.empty()) return;
  for (const Term &t : H.terms) {
    int in[4], ext[4], ki = 0, ko = 0;
    for (int i = 0; i < t.n; ++i) {
      const bool inside = left ? (H.site_of(t.e[i]) < bond) : (H.site_of(t.e[i]) >= bond);
      if (inside)
        in[ki++] = t.e[i];
      else
        ext[ko++] = t.e[i];
    }
    if (ki == 0 || ko == 0) continue;
    if (left && t.n == 4 && ki == 3) continue;
    if (!left && ki != 1) continue;
    const uint64_t k = make_key(K_X, ext, ko);
    if (!wanted.count(k)) continue;
    out[k][make_key(K_N, in, ki)] += t.c;
  }
}

static QN combo_delta(const Hamiltonian &H, bool left, uint64_t key) {
  // decode external list
  int e[4];
  const int n = key_n(key);
  for (int i = 0; i < n; ++i) e[i] = int((key >> (8 + 13 * i)) & 8191) - 1;
  const QN qe = q_sum(H, e, n);
  return left ? QN() - qe : qe;
}

// Materialise combos X (already laid out) from the stored operators of env.
static void materialize(Device *dev, OpSet &X, const OpSet &env, const Content &content) {
  for (size_t g = 0; g < X.groups.size(); ++g) {
    const Group &GX = X.groups[g];
    if (GX.size == 0 || GX.n_ops == 0) continue;
    auto ge = env.gidx.find(GX.delta.key());
    if (ge == env.gidx.end()) continue;
    const Group &GE = env.groups[ge->second];
    MDMRG_REQUIRE(GE.size == GX.size, -4, "materialize: layout mismatch");
    std::vector<double> C(size_t(GX.n_ops) * GE.n_ops, 0.0);
    bool any = false;
    for (auto &kv : X.ops) {
      if (kv.second.first != int(g)) continue;
      auto ct = content.find(kv.first);
      if (ct == content.end()) continue;
      for (auto &src : ct->second) {
        auto se = env.ops.find(src.first);
        if (se == env.ops.end()) continue;
        MDMRG_REQUIRE(se->second.first == ge->second, -4, "materialize: source in wrong group");
        C[size_t(kv.second.second) * GE.n_ops + se->second.second] += src.second;
        any = true;
      }
    }
    if (!any) continue;
    double *dC = (double *)dev_alloc(dev, sizeof(double) * C.size());
    dev_h2d(dev, dC, C.data(), sizeof(double) * C.size());
    GemmPlan plan;
    GSeg s{};
    s.a_off = 0;
    s.b_off = GE.base;
    s.alpha = 1.0;
    s.k = GE.n_ops;
    s.lda = GE.n_ops;
    s.ldb = int32_t(GE.size);
    MDMRG_REQUIRE(GE.size < (int64_t(1) << 31), -6, "operator too large for int32 leading dimension");
    s.a_slot = 0;
    s.b_slot = 2;
    s.flags = 0;
    plan.segs.push_back(s);
    GOut o{};
    o.c_off = GX.base;
    o.m = GX.n_ops;
    o.n = int32_t(GX.size);
    o.ldc = int32_t(GX.size);
    o.seg_begin = 0;
    o.seg_count = 1;
    o.c_slot = 1;
    o.accumulate = 0;
    plan.outs.push_back(o);
    DevPlan *dp = dev_plan_upload(dev, plan);
    Bases b{};
    b.p[0] = dC;
    b.p[1] = X.arena;
    b.p[2] = env.arena;
    for (int i = 3; i < kSlots; ++i) b.p[i] = dC;
    dev_gemm_run(dev, dp, b);
    dev_plan_free(dev, dp);
    dev_free(dev, dC);
  }
}

// ------------------------------------------------------- two-phase planner
// split_stride > 0 enables split-K of the accumulation phase: outputs are
// the blocks of one buffer of split_stride elements; their K-concatenated
// segment lists are cut into plan.n_split contiguous groups written to
// partial copies (slot 7) and summed by a fixed-order reduction.
static void build_two_phase(std::vector<PairTask> &tasks, const std::vector<OutBlk> &outs, int64_t limit,
                            TwoPhasePlan &plan, Device *dev, int64_t split_stride = 0) {
  std::stable_sort(tasks.begin(), tasks.end(), [](const PairTask &a, const PairTask &b) { return a.out < b.out; });
  plan.scratch = 0;
  {
    // algorithmic bytes: every distinct operand block read once, every
    // output block written once
    // (slot, element offset) of a block, packed: offsets stay below 2^56
    auto bkey = [](const Ref &r) { return (uint64_t(r.slot) << 56) ^ uint64_t(r.off); };
    std::unordered_set<uint64_t> seen;
    seen.reserve(tasks.size() * 2);
    double elems = 0.0;
    for (const PairTask &t : tasks) {
      if (!t.idA && seen.insert(bkey(t.A)).second) elems += double(t.m) * t.k1;
      if (seen.insert(bkey(t.X)).second) elems += double(t.k1) * t.k2;
      if (!t.idB && seen.insert(bkey(t.B)).second) elems += double(t.k2) * t.n;
    }
    std::vector<char> so(outs.size(), 0);
    for (const PairTask &t : tasks)
      if (!so[t.out]) {
        so[t.out] = 1;
        elems += double(outs[t.out].m) * outs[t.out].n;
      }
    plan.bytes += 8.0 * elems;
  }
  struct TKey {
    int order;
    int xs;
    int64_t xo;
    int os;
    int64_t oo;
    int tr;
    bool operator==(const TKey &o) const {
      return order == o.order && xs == o.xs && xo == o.xo && os == o.os && oo == o.oo && tr == o.tr;
    }
  };
  struct TKeyHash {
    size_t operator()(const TKey &k) const {
      uint64_t h = uint64_t(k.xo) * 0x9E3779B97F4A7C15ull;
      h ^= (uint64_t(k.oo) + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2));
      h ^= uint64_t(k.order | (k.xs << 2) | (k.os << 6) | (k.tr << 10)) * 0xBF58476D1CE4E5B9ull;
      return size_t(h ^ (h >> 31));
    }
  };
  size_t i = 0;
  while (i < tasks.size()) {
    GemmPlan p1, p2;
    std::unordered_map<TKey, int64_t, TKeyHash> tmap;
    int64_t used = 0;
    std::vector<std::vector<GSeg>> per_out;
    std::vector<int32_t> out_ids;
    int cur_out = -1;
    size_t j = i;
    for (; j < tasks.size(); ++j) {
      const PairTask &t = tasks[j];
      // chunk boundary only between outputs
      if (t.out != cur_out && used > limit && !out_ids.empty()) break;
      if (t.out != cur_out) {
        cur_out = t.out;
        out_ids.push_back(t.out);
        per_out.emplace_back();
      }
      std::vector<GSeg> &segs = per_out.back();
      GSeg s{};
      s.alpha = t.alpha;
      auto refA = [&](GSeg &g, const Ref &r, bool tr) {
        g.a_slot = uint8_t(r.slot);
        g.a_off = r.off;
        g.lda = r.ld;
        if (tr) g.flags |= SEG_TA;
      };
      auto refB = [&](GSeg &g, const Ref &r, bool tr) {
        g.b_slot = uint8_t(r.slot);
        g.b_off = r.off;
        g.ldb = r.ld;
        if (tr) g.flags |= SEG_TB;
      };
      if (t.idA && t.idB) {
        s.flags = SEG_AID;
        s.a_slot = 0;
        s.a_off = 0;
        s.lda = 0;
        refB(s, t.X, false);
        s.k = t.k1;
        segs.push_back(s);
        continue;
      }
      if (t.idA) {
        refA(s, t.X, false);
        refB(s, t.B, t.tB);
        s.k = t.k2;
        p2.flop += 2.0 * t.m * t.n * t.k2;
        plan.hist_add(t.m, t.n, 2.0 * t.m * t.n * t.k2);
        segs.push_back(s);
        continue;
      }
      if (t.idB) {
        refA(s, t.A, t.tA);
        refB(s, t.X, false);
        s.k = t.k1;
        p2.flop += 2.0 * t.m * t.n * t.k1;
        plan.hist_add(t.m, t.n, 2.0 * t.m * t.n * t.k1);
        segs.push_back(s);
        continue;
      }
      const double c_lr = double(t.m) * t.k1 * t.k2 + double(t.m) * t.k2 * t.n;  // (A X) B
      const double c_rl = double(t.k1) * t.k2 * t.n + double(t.m) * t.k1 * t.n;  // A (X B)
      if (c_rl <= c_lr) {
        TKey key{1, t.X.slot, t.X.off, t.B.slot, t.B.off, int(t.tB)};
        auto it = tmap.find(key);
        int64_t toff;
        if (it == tmap.end()) {
          toff = used;
          used += (int64_t(t.k1) * t.n + 7) / 8 * 8;
          tmap[key] = toff;
          GSeg s1{};
          s1.alpha = 1.0;
          refA(s1, t.X, false);
          refB(s1, t.B, t.tB);
          s1.k = t.k2;
          GOut o{};
          o.c_off = toff;
          o.m = t.k1;
          o.n = t.n;
          o.ldc = t.n;
          o.seg_begin = int32_t(p1.segs.size());
          o.seg_count = 1;
          o.c_slot = 2;
          o.accumulate = 0;
          p1.segs.push_back(s1);
          p1.outs.push_back(o);
          p1.flop += 2.0 * t.k1 * t.n * t.k2;
          plan.hist_add(t.k1, t.n, 2.0 * t.k1 * t.n * t.k2);
        } else {
          toff = it->second;
        }
        refA(s, t.A, t.tA);
        refB(s, Ref{2, toff, t.n}, false);
        s.k = t.k1;
        p2.flop += 2.0 * t.m * t.n * t.k1;
        plan.hist_add(t.m, t.n, 2.0 * t.m * t.n * t.k1);
      } else {
        TKey key{0, t.X.slot, t.X.off, t.A.slot, t.A.off, int(t.tA)};
        auto it = tmap.find(key);
        int64_t toff;
        if (it == tmap.end()) {
          toff = used;
          used += (int64_t(t.m) * t.k2 + 7) / 8 * 8;
          tmap[key] = toff;
          GSeg s1{};
          s1.alpha = 1.0;
          refA(s1, t.A, t.tA);
          refB(s1, t.X, false);
          s1.k = t.k1;
          GOut o{};
          o.c_off = toff;
          o.m = t.m;
          o.n = t.k2;
          o.ldc = t.k2;
          o.seg_begin = int32_t(p1.segs.size());
          o.seg_count = 1;
          o.c_slot = 2;
          o.accumulate = 0;
          p1.segs.push_back(s1);
          p1.outs.push_back(o);
          p1.flop += 2.0 * t.m * t.k2 * t.k1;
          plan.hist_add(t.m, t.k2, 2.0 * t.m * t.k2 * t.k1);
        } else {
          toff = it->second;
        }
        refA(s, Ref{2, toff, t.k2}, false);
        refB(s, t.B, t.tB);
        s.k = t.k2;
        p2.flop += 2.0 * t.m * t.n * t.k2;
        plan.hist_add(t.m, t.n, 2.0 * t.m * t.n * t.k2);
      }
      segs.push_back(s);
    }
    // split-K factor: enough workgroup tiles to fill the chip
    int S = 1;
    if (split_stride > 0) {
      int64_t tiles = 0;
      size_t maxseg = 0;
      for (size_t q = 0; q < out_ids.size(); ++q) {
        const OutBlk &ob = outs[out_ids[q]];
        tiles += int64_t((ob.m + 63) / 64) * ((ob.n + 63) / 64);
        maxseg = std::max(maxseg, per_out[q].size());
      }
      // about 16384 workgroup tiles (several waves of workgroups per CU, so
      // the tail of the launch is short), at most 32 partial copies
      S = int(std::min<int64_t>(std::max<int64_t>(1, 16384 / std::max<int64_t>(tiles, 1)), 32));
      S = int(std::min<size_t>(size_t(S), std::max<size_t>(maxseg, 1)));
      plan.n_split = std::max(plan.n_split, S);
    }
    std::vector<int64_t> roff;
    std::vector<int32_t> rlen;
    for (size_t q = 0; q < out_ids.size(); ++q) {
      const OutBlk &ob = outs[out_ids[q]];
      const std::vector<GSeg> &sv = per_out[q];
      if (S == 1) {
        GOut o{};
        o.c_off = ob.off;
        o.m = ob.m;
        o.n = ob.n;
        o.ldc = ob.ld;
        o.seg_begin = int32_t(p2.segs.size());
        o.seg_count = int32_t(sv.size());
        o.c_slot = uint8_t(ob.slot);
        o.accumulate = 1;
        p2.segs.insert(p2.segs.end(), sv.begin(), sv.end());
        p2.outs.push_back(o);
        continue;
      }
      // contiguous groups balanced by K; every (block, group) is written
      // (empty groups write zeros) so no stale partial survives a chunk
      double ktot = 0.0;
      for (const GSeg &g : sv) ktot += g.k + 4.0;
      size_t pos = 0;
      double acc = 0.0;
      for (int q2 = 0; q2 < S; ++q2) {
        const double goal = ktot * (q2 + 1) / S;
        GOut o{};
        o.c_off = int64_t(q2) * split_stride + ob.off;
        o.m = ob.m;
        o.n = ob.n;
        o.ldc = ob.ld;
        o.seg_begin = int32_t(p2.segs.size());
        o.c_slot = 7;
        o.accumulate = 0;
        while (pos < sv.size() && (acc < goal - 1e-9 || q2 == S - 1)) {
          p2.segs.push_back(sv[pos]);
          acc += sv[pos].k + 4.0;
          ++pos;
        }
        o.seg_count = int32_t(p2.segs.size()) - o.seg_begin;
        p2.outs.push_back(o);
      }
      MDMRG_REQUIRE(ob.ld == ob.n, -4, "split-K needs packed output blocks");
      roff.push_back(ob.off);
      rlen.push_back(ob.m * ob.n);
    }
    plan.n_gemm += int64_t(p1.segs.size() + p2.segs.size());
    plan.flop += p1.flop + p2.flop;
    plan.bytes += 16.0 * double(used);  // intermediates written and read back
    plan.scratch = std::max(plan.scratch, used);
    Chunk ch;
    ch.p1 = p1.outs.empty() ? nullptr : dev_plan_upload(dev, p1);
    ch.p2 = p2.outs.empty() ? nullptr : dev_plan_upload(dev, p2);
    if (S > 1) ch.red = dev_reduce_upload(dev, roff, rlen, S, split_stride);
    plan.chunks.push_back(ch);
    i = j;
  }
}

void Context::ensure_scratch(int64_t n) {
  if (n <= T_scratch_n) return;
  release_graphs();  // captured graphs hold the old address
  if (T_scratch) dev_free(dev, T_scratch);
  T_scratch = (double *)dev_alloc(dev, sizeof(double) * std::max<int64_t>(n, 1));
  T_scratch_n = n;
}

void Context::run_plan(const TwoPhasePlan &p, Bases &b, int tag, int prec) {
  // phase-1 launches of an H_eff product are timed under tag 5
  b.p[2] = T_scratch;
  if (p.n_split > 1) b.p[7] = P_scratch;
  for (auto &c : p.chunks) {
    if (c.p1) dev_gemm_run(dev, c.p1, b, tag == 1 ? 5 : tag, prec);
    if (c.p2) dev_gemm_run(dev, c.p2, b, tag, prec);
    if (c.red) dev_reduce_run(dev, c.red, P_scratch, b.p[1], prec);
  }
}

// ------------------------------------------------------------- boundaries
std::unique_ptr<OpSet> Context::env_boundary(bool left, int bond) {
  auto S = std::make_unique<OpSet>();
  S->bond = &bonds[bond];
  if (left)
    need_left(ham, bond, *S);
  else
    need_right(ham, bond, *S);
  S->layout(dev);  // all zero: empty block, H = 0, no operators act
  return S;
}

// Renormalise recipes (items per new operator) into the new OpSet.
// left: new(a'',c'') += sum alpha A(a,s,a'')^T X(a,c) A(c,t,c'')
// right: new(b'',c'') += sum alpha B(b'',s,b) X(b,c) B(c'',t,c)^T
struct Recipe {
  std::map<OpRef, SiteItem> items;
};

static void add_item(Recipe &r, OpRef ref, const std::vector<double> &M, int parity, double scale) {
  auto it = r.items.find(ref);
  if (it == r.items.end()) {
    SiteItem si;
    si.M.assign(M.size(), 0.0);
    si.parity = parity;
    it = r.items.emplace(ref, si).first;
  }
  for (size_t i = 0; i < M.size(); ++i) it->second.M[i] += scale * M[i];
}

static void renorm_execute(Context &C, bool left, int site, OpSet &Bp, const OpSet &env, const OpSet *combo,
                           const std::unordered_map<uint64_t, Recipe> &recipes,
                           const std::vector<uint64_t> *keys = nullptr) {
  const Hamiltonian &H = C.ham;
  const int d = H.d;
  const Bond &bo = C.bonds[left ? site : site + 1];  // old block bond
  const Bond &bn = C.bonds[left ? site + 1 : site];  // new block bond
  const SiteTensor &T = C.A[site];
  std::vector<PairTask> tasks;
  std::vector<OutBlk> outs;
  GemmPlan direct;  // identity X: Y += alpha op(A) op(B), one GEMM each
  for (uint64_t key : keys ? *keys : Bp.order) {
    auto rit = recipes.find(key);
    if (rit == recipes.end()) continue;
    const auto [g, idx] = Bp.ops.at(key);
    const Group &G = Bp.groups[g];
    for (size_t p = 0; p < G.row.size(); ++p) {
      const int rn = G.row[p], cn = G.col[p];
      const int64_t yoff = G.base + int64_t(idx) * G.size + G.poff[p];
      const int out_id = int(outs.size());
      bool used = false;
      std::vector<GSeg> dsegs;
      for (auto &it : rit->second.items) {
        const OpRef &ref = it.first;
        const SiteItem &si = it.second;
        const OpSet *src = ref.src == 1 ? &env : ref.src == 2 ? combo : nullptr;
        if (ref.src && (!src || !src->has(ref.key))) continue;
        const int pX = ref.src == 0 ? 0 : key_parity(ref.key);
        for (int s = 0; s < d; ++s)
          for (int t = 0; t < d; ++t) {
            const double m = si.M[s * d + t];
            if (m == 0.0) continue;
            int ro, co, ia, ic;
            if (left) {
              ro = bo.find(bn.qn[rn] - H.q_of_state(s));
              co = bo.find(bn.qn[cn] - H.q_of_state(t));
              if (ro < 0 || co < 0) continue;
              ia = T.find(ro, s, rn);
              ic = T.find(co, t, cn);
            } else {
              ro = bo.find(bn.qn[rn] + H.q_of_state(s));
              co = bo.find(bn.qn[cn] + H.q_of_state(t));
              if (ro < 0 || co < 0) continue;
              ia = T.find(rn, s, ro);
              ic = T.find(cn, t, co);
            }
            if (ia < 0 || ic < 0) continue;
            int64_t xoff = -1;
            if (ref.src == 0) {
              if (ro != co) continue;
            } else {
              int row = -1;
              xoff = src->block(ref.key, co, &row);
              if (xoff < 0 || row != ro) continue;
            }
            double sign = 1.0;
            if (left) {
              if ((si.parity & 1) && bo.qn[co].parity()) sign = -1.0;
            } else {
              if ((pX & 1) && parity_of_state(t)) sign = -1.0;
            }
            const int mro = bo.dim[ro], mco = bo.dim[co], mrn = bn.dim[rn], mcn = bn.dim[cn];
            Ref Ar, Br;
            bool tA, tB;
            if (left) {  // A(ro,s,rn)^T [mrn x mro], B = A(co,t,cn) [mco x mcn]
              Ar = Ref{6, T.off[ia], mrn};
              tA = true;
              Br = Ref{6, T.off[ic], mcn};
              tB = false;
            } else {  // B(rn,s,ro) [mrn x mro], B(cn,t,co)^T [mco x mcn]
              Ar = Ref{6, T.off[ia], mro};
              tA = false;
              Br = Ref{6, T.off[ic], mco};
              tB = true;
            }
            used = true;
            if (ref.src == 0) {
              GSeg s1{};
              s1.alpha = m * sign;
              s1.a_slot = 6;
              s1.a_off = Ar.off;
              s1.lda = Ar.ld;
              s1.b_slot = 6;
              s1.b_off = Br.off;
              s1.ldb = Br.ld;
              s1.flags = uint8_t((tA ? SEG_TA : 0) | (tB ? SEG_TB : 0));
              s1.k = mro;
              dsegs.push_back(s1);
              direct.flop += 2.0 * mrn * mcn * mro;
              continue;
            }
            PairTask pt{};
            pt.out = out_id;
            pt.alpha = m * sign;
            pt.A = Ar;
            pt.tA = tA;
            pt.B = Br;
            pt.tB = tB;
            pt.X = Ref{ref.src == 1 ? 3 : 5, xoff, mco};
            pt.m = mrn;
            pt.k1 = mro;
            pt.k2 = mco;
            pt.n = mcn;
            tasks.push_back(pt);
          }
      }
      if (!used) continue;
      outs.push_back(OutBlk{1, yoff, bn.dim[rn], bn.dim[cn], bn.dim[cn]});
      if (!dsegs.empty()) {
        GOut o{};
        o.c_off = yoff;
        o.m = bn.dim[rn];
        o.n = bn.dim[cn];
        o.ldc = o.n;
        o.c_slot = 1;
        o.accumulate = 1;
        o.seg_begin = int32_t(direct.segs.size());
        o.seg_count = int32_t(dsegs.size());
        direct.segs.insert(direct.segs.end(), dsegs.begin(), dsegs.end());
        direct.outs.push_back(o);
      }
    }
  }
  TwoPhasePlan plan;
  // intermediates of the renormalisation products in passes of at most the
  // combination limit, so that an environment build holds little besides
  // the old and the new block
  build_two_phase(tasks, outs, std::min(C.scratch_limit, C.ren_combo_limit), plan, C.dev);
  if (!direct.outs.empty()) {
    Chunk ch;
    ch.p2 = dev_plan_upload(C.dev, direct);
    plan.chunks.push_back(ch);
    plan.flop += direct.flop;
  }
  C.ensure_scratch(plan.scratch);
  if (C.ren_prec == 0) {
    Bases b{};
    for (int i = 0; i < kSlots; ++i) b.p[i] = Bp.arena;
    b.p[1] = Bp.arena;
    b.p[3] = env.arena;
    b.p[5] = combo && combo->arena ? combo->arena : Bp.arena;
    b.p[6] = T.data;
    C.run_plan(plan, b, 2);
  } else {
    // split-precision renormalisation: the same plan on FP32 copies of the
    // source operators and of the site tensor (FP32 or 3xBF16 products, FP32
    // accumulation); the new operators are stored back as FP64 masters, so
    // every later step reads them as usual.  The new arena is all zero at
    // this point, so converting the FP32 result overwrites nothing.
    DevVecs tmp(C.dev);
    auto f32 = [&](const double *src, int64_t n) -> float * {
      float *f = reinterpret_cast<float *>(tmp.get((std::max<int64_t>(1, n) + 1) / 2));
      if (n > 0) dev_d2f(C.dev, src, f, n);
      return f;
    };
    float *env32 = f32(env.arena, env.arena_size);
    float *T32 = f32(T.data, T.size);
    float *combo32 = combo && combo->arena ? f32(combo->arena, combo->arena_size) : nullptr;
    float *out32 = reinterpret_cast<float *>(tmp.get((std::max<int64_t>(1, Bp.arena_size) + 1) / 2));
    dev_zero(C.dev, out32, sizeof(float) * std::max<int64_t>(1, Bp.arena_size));
    Bases b{};
    for (int i = 0; i < kSlots; ++i) b.p[i] = reinterpret_cast<double *>(out32);
    b.p[3] = reinterpret_cast<double *>(env32);
    if (combo32) b.p[5] = reinterpret_cast<double *>(combo32);
    b.p[6] = reinterpret_cast<double *>(T32);
    C.run_plan(plan, b, 2, C.ren_prec);
    dev_f2d(C.dev, out32, Bp.arena, Bp.arena_size);
    dev_sync(C.dev);  // the FP32 copies are freed at scope end
  }
  plan.release(C.dev);
}

// Elements of one block operator with quantum-number shift delta on bond b
// (the group size of OpSet::layout).
static int64_t op_elems(const Bond &b, QN delta) {
  int64_t n = 0;
  for (size_t c = 0; c < b.qn.size(); ++c) {
    const int r = b.find(b.qn[c] + delta);
    if (r >= 0) n += int64_t(b.dim[r]) * b.dim[c];
  }
  return n;
}

// Renormalise the recipes of the new block Bp in batches of its operators.
// The on-the-fly combinations of the old block's operators that a batch
// reads (a3: one grouped GEMM per shift group) are formed for that batch
// only and released after its products, so their storage stays below
// `limit` doubles (or one batch's need) however many operators the block
// holds: at large D a block carries thousands of operators of tens of MB.
// The split-precision forms convert the whole new block once, so they run
// as a single batch.
static void renorm_batched(Context &C, bool left, int site, OpSet &Bp, const OpSet &env, int content_bond,
                           const std::unordered_map<uint64_t, Recipe> &rec) {
  const Hamiltonian &H = C.ham;
  const int64_t limit = C.ren_prec == 0 ? C.ren_combo_limit : std::numeric_limits<int64_t>::max();
  std::vector<std::vector<uint64_t>> batches(1);
  std::vector<std::set<uint64_t>> wanted(1);
  int64_t acc = 0;
  for (uint64_t key : Bp.order) {
    auto it = rec.find(key);
    if (it == rec.end()) continue;
    for (int pass = 0; pass < 2; ++pass) {
      int64_t need = 0;
      for (auto &item : it->second.items)
        if (item.first.src == 2 && !wanted.back().count(item.first.key))
          need += op_elems(*env.bond, combo_delta(H, left, item.first.key));
      if (pass == 0 && acc + need > limit && !batches.back().empty()) {
        batches.emplace_back();
        wanted.emplace_back();
        acc = 0;
        continue;
      }
      acc += need;
      for (auto &item : it->second.items)
        if (item.first.src == 2) wanted.back().insert(item.first.key);
      batches.back().push_back(key);
      break;
    }
  }
  // content of every combination read by any batch (host only), in one pass
  // over the terms; each batch materialises its own keys from it
  std::set<uint64_t> all;
  for (auto &w : wanted) all.insert(w.begin(), w.end());
  Content content;
  combo_content(H, left, content_bond, all, content);
  for (size_t b = 0; b < batches.size(); ++b) {
    if (batches[b].empty()) continue;
    std::unique_ptr<OpSet> X;
    if (!wanted[b].empty()) {
      X = std::make_unique<OpSet>();
      X->bond = env.bond;
      for (uint64_t k : wanted[b]) X->add(k, combo_delta(H, left, k));
      X->layout(C.dev);
      materialize(C.dev, *X, env, content);
    }
    renorm_execute(C, left, site, Bp, env, X.get(), rec, &batches[b]);
    if (X) X->release(C.dev);
  }
}

// L(bond site) + site -> L(bond site+1), with A[site] a left isometry
std::unique_ptr<OpSet> Context::renorm_left(const OpSet &L, int site) {
  const Hamiltonian &H = ham;
  const int d = H.d;
  auto Lp = std::make_unique<OpSet>();
  Lp->bond = &bonds[site + 1];
  need_left(H, site + 1, *Lp);
  Lp->layout(dev);
  std::unordered_map<uint64_t, Recipe> rec;
  std::vector<double> I(d * d, 0.0);
  for (int s = 0; s < d; ++s) I[s * d + s] = 1.0;
  const uint64_t kH = make_key(K_H, nullptr, 0);
  const OpRef ident{0, ident_key()};
  // H_{L'}
  add_item(rec[kH], OpRef{1, kH}, I, 0, 1.0);
  std::set<std::pair<OpRef, uint64_t>> seen;  // (source, site-op list) pairs already added
  auto add_set = [&](uint64_t newkey, OpRef src, const int *es, int ks) {
    const uint64_t sk = make_key(K_N, es, ks);
    if (!seen.insert({src, sk ^ (newkey * 0x9E3779B97F4A7C15ull)}).second) return;
    add_item(rec[newkey], src, H.site_matrix(site, es, ks), ks & 1, 1.0);
  };
  for (const Term &t : H.terms) {
    Parts p;
    split(H, t, site, p);  // 0: L, 1: site, 2,3: outside
    const int kout = p.k[2] + p.k[3];
    int ext[4], ke = 0;
    for (int i = 0; i < p.k[2]; ++i) ext[ke++] = p.e[2][i];
    for (int i = 0; i < p.k[3]; ++i) ext[ke++] = p.e[3][i];
    if (kout == 0 && p.k[1] >= 1) {
      if (p.k[0] == 0) {
        add_item(rec[kH], ident, H.site_matrix(site, p.e[1], p.k[1]), 0, t.c);
      } else {
        const uint64_t kk = (t.n == 4 && p.k[0] == 3) ? make_key(K_C, p.e[1], p.k[1]) : make_key(K_X, p.e[1], p.k[1]);
        add_set(kH, OpRef{(t.n == 4 && p.k[0] == 3) ? 1 : 2, kk}, p.e[1], p.k[1]);
      }
    }
    // S^{L'}_y: two-body terms with three operators in L' and one outside
    if (t.n == 4 && kout == 1 && p.k[0] + p.k[1] == 3) {
      const uint64_t nk = make_key(K_C, ext, 1);
      if (!Lp->has(nk)) continue;
      if (p.k[0] == 3) {
        add_set(nk, OpRef{1, nk}, nullptr, 0);
      } else if (p.k[0] >= 1) {
        int K[4], kk = 0;
        for (int i = 0; i < p.k[1]; ++i) K[kk++] = p.e[1][i];
        K[kk++] = ext[0];
        add_set(nk, OpRef{2, make_key(K_X, K, kk)}, p.e[1], p.k[1]);
      } else {
        add_item(rec[nk], ident, H.site_matrix(site, p.e[1], p.k[1]), p.k[1] & 1, t.c);
      }
    }
  }
  // normal operators
  for (uint64_t key : Lp->order) {
    if (key_kind(key) != K_N) continue;
    const int n = key_n(key);
    int e[4];
    for (int i = 0; i < n; ++i) e[i] = int((key >> (8 + 13 * i)) & 8191) - 1;
    int kin = 0;
    while (kin < n && H.site_of(e[kin]) < site) ++kin;
    if (kin == n) {
      add_item(rec[key], OpRef{1, key}, I, 0, 1.0);
    } else if (kin == 0) {
      add_item(rec[key], ident, H.site_matrix(site, e, n), n & 1, 1.0);
    } else {
      add_item(rec[key], OpRef{1, make_key(K_N, e, kin)}, H.site_matrix(site, e + kin, n - kin), (n - kin) & 1, 1.0);
    }
  }
  // with the combos of L that the recipes read, formed per batch
  renorm_batched(*this, true, site, *Lp, L, site, rec);
  return Lp;
}

// R(bond site+1) + site -> R(bond site), with A[site] a right isometry
std::unique_ptr<OpSet> Context::renorm_right(const OpSet &R, int site) {
  const Hamiltonian &H = ham;
  const int d = H.d;
  auto Rp = std::make_unique<OpSet>();
  Rp->bond = &bonds[site];
  need_right(H, site, *Rp);
  Rp->layout(dev);
  std::unordered_map<uint64_t, Recipe> rec;
  std::vector<double> I(d * d, 0.0);
  for (int s = 0; s < d; ++s) I[s * d + s] = 1.0;
  const uint64_t kH = make_key(K_H, nullptr, 0);
  const OpRef ident{0, ident_key()};
  add_item(rec[kH], OpRef{1, kH}, I, 0, 1.0);
  std::set<std::pair<OpRef, uint64_t>> seen;
  auto add_set = [&](uint64_t newkey, OpRef src, const int *es, int ks) {
    const uint64_t sk = make_key(K_N, es, ks);
    if (!seen.insert({src, sk ^ (newkey * 0x9E3779B97F4A7C15ull)}).second) return;
    add_item(rec[newkey], src, H.site_matrix(site, es, ks), ks & 1, 1.0);
  };
  for (const Term &t : H.terms) {
    // parts relative to the new block: outside (< site), site, R (> site)
    int out[4], sp[4], ko = 0, ks = 0, kr = 0;
    for (int i = 0; i < t.n; ++i) {
      const int st = H.site_of(t.e[i]);
      if (st < site)
        out[ko++] = t.e[i];
      else if (st == site)
        sp[ks++] = t.e[i];
      else
        ++kr;
    }
    if (ks + kr == 0) continue;
    if (ko == 0) {  // H_{R'}
      if (ks == 0) continue;  // in H_R
      if (kr == 0) {
        add_item(rec[kH], ident, H.site_matrix(site, sp, ks), 0, t.c);
      } else {
        const bool stored = ks <= 2;
        add_set(kH, OpRef{stored ? 1 : 2, make_key(stored ? K_C : K_X, sp, ks)}, sp, ks);
      }
      continue;
    }
    if (ko > 2) continue;
    const uint64_t nk = make_key(K_C, out, ko);
    if (!Rp->has(nk)) continue;
    if (kr == 0) {
      add_item(rec[nk], ident, H.site_matrix(site, sp, ks), ks & 1, t.c);
      continue;
    }
    int K[4], kk = 0;
    for (int i = 0; i < ko; ++i) K[kk++] = out[i];
    for (int i = 0; i < ks; ++i) K[kk++] = sp[i];
    const bool stored = kk <= 2;
    add_set(nk, OpRef{stored ? 1 : 2, make_key(stored ? K_C : K_X, K, kk)}, sp, ks);
  }
  for (uint64_t key : Rp->order) {
    if (key_kind(key) != K_N) continue;
    int e = int((key >> 8) & 8191) - 1;
    if (H.site_of(e) == site)
      add_item(rec[key], ident, H.site_matrix(site, &e, 1), 1, 1.0);
    else
      add_item(rec[key], OpRef{1, key}, I, 0, 1.0);
  }
  renorm_batched(*this, false, site, *Rp, R, site + 1, rec);
  return Rp;
}

// ------------------------------------------------------------- layout
PsiLayout Context::make_layout(int l) const {
  PsiLayout L;
  const Bond &ba = bonds[l], &bb = bonds[l + 2];
  const int d = ham.d;
  for (size_t a = 0; a < ba.qn.size(); ++a)
    for (int s1 = 0; s1 < d; ++s1)
      for (int s2 = 0; s2 < d; ++s2) {
        const QN q = ba.qn[a] + ham.q_of_state(s1) + ham.q_of_state(s2);
        const int b = bb.find(q);
        if (b < 0 || ba.dim[a] == 0 || bb.dim[b] == 0) continue;
        PsiBlk pb{int(a), s1, s2, b, ba.dim[a], bb.dim[b], L.n_elem};
        L.idx[PsiLayout::key(int(a), s1, s2, b)] = int(L.blk.size());
        L.blk.push_back(pb);
        L.n_elem += int64_t(pb.m) * pb.n;
      }
  return L;
}

// ------------------------------------------------------------- prepare
void Context::release_graphs() {
  dev_graph_free(dev, graph64);
  dev_graph_free(dev, graph32);
  dev_graph_free(dev, graphbf3);
  dev_graph_free(dev, graphbf6);
  graph64 = graph32 = graphbf3 = graphbf6 = nullptr;
  eager64 = eager32 = eagerbf3 = eagerbf6 = 0;
}

void Context::set_graph(bool on) {
  use_graph = on;
  if (!on) {
    release_graphs();
    for (double **p : {&xg, &yg}) {
      if (*p) dev_free(dev, *p);
      *p = nullptr;
    }
    xg_n = 0;
  }
}

void Context::release_bond() {
  release_graphs();
  for (float **p : {&L32, &R32, &Lx32, &Rx32, &x32, &y32}) {
    if (*p) dev_free(dev, *p);
    *p = nullptr;
  }
  heff.release(dev);
  if (diag) dev_diag_free(dev, diag);
  diag = nullptr;
  if (Lx) Lx->release(dev);
  if (Rx) Rx->release(dev);
  Lx.reset();
  Rx.reset();
  cur = -1;
}

void Context::reset_envs() {
  release_bond();
  for (auto &e : Lenv)
    if (e) e->release(dev);
  for (auto &e : Renv)
    if (e) e->release(dev);
  Lenv.clear();
  Renv.clear();
}

Context::~Context() {
  if (!dev) return;
  try {
    reset_envs();
    for (auto &t : A)
      if (t.data) dev_free(dev, t.data);
    if (T_scratch) dev_free(dev, T_scratch);
    if (P_scratch) dev_free(dev, P_scratch);
    set_graph(false);
    dev_sync(dev);
  } catch (...) {
  }
  dev_destroy(dev);
}

void Context::prepare(int l) {
  MDMRG_REQUIRE(have_ham && have_mps, -4, "prepare_bond: Hamiltonian and MPS required");
  const int n = ham.n;
  MDMRG_REQUIRE(l >= 0 && l + 1 < n, -1, "prepare_bond: bond out of range");
  double t0 = wall_seconds();
  if (int(Lenv.size()) != n + 1) {
    Lenv.resize(n + 1);
    Renv.resize(n + 1);
  }
  auto drop = [&](std::unique_ptr<OpSet> &e) {
    if (e) e->release(dev);
    e.reset();
  };
  bool built = false;
  const bool verbose = std::getenv("MDMRG_VERBOSE") != nullptr;
  // the builds start from the nearest existing block on each side
  int li = l, ri = l + 2;
  while (li > 0 && !Lenv[li]) --li;
  while (ri < n && !Renv[ri]) ++ri;
  // blocks kept at this bond (MDMRG_OPT_KEEP_ENVS): 1 every block built;
  // 0 this bond's and one step either way (L at l-1, l; R at l+2, l+3);
  // 2 a walk to the right (L at l; every R at bonds >= l+2, so each later
  // step finds its right block); 3 one step to the right (L at l; R at l+2,
  // l+3).  Blocks outside the set are dropped before any build, and each
  // source block once the next one is built.
  auto keepL = [&](int j) { return keep_envs == 1 || j == l || (keep_envs == 0 && j == l - 1); };
  auto keepR = [&](int j) {
    return keep_envs == 1 || j == l + 2 || (keep_envs == 2 && j > l + 2) ||
           ((keep_envs == 0 || keep_envs == 3) && j == l + 3);
  };
  for (int j = 0; j <= n; ++j) {
    if (!keepL(j) && j != li) drop(Lenv[j]);
    if (!keepR(j) && j != ri) drop(Renv[j]);
  }
  // right blocks first: they carry the complementary operators with two
  // outside indices, the largest blocks of the chain, and are built while no
  // left block of this bond holds memory yet
  if (!Renv[l + 2]) {
    built = true;
    if (!Renv[ri]) Renv[ri] = env_boundary(false, ri);
    for (int i = ri - 1; i >= l + 2; --i) {
      Renv[i] = renorm_right(*Renv[i + 1], i);
      if (verbose) fprintf(stderr, "[mdmrg] right block at bond %d built\n", i);
      if (!keepR(i + 1)) drop(Renv[i + 1]);
    }
  }
  if (!Lenv[l]) {
    built = true;
    if (!Lenv[li]) Lenv[li] = env_boundary(true, li);
    for (int i = li; i < l; ++i) {
      Lenv[i + 1] = renorm_left(*Lenv[i], i);
      if (verbose) fprintf(stderr, "[mdmrg] left block at bond %d built\n", i + 1);
      if (!keepL(i)) drop(Lenv[i]);
    }
  }
  if (!keepL(li)) drop(Lenv[li]);
  if (!keepR(ri)) drop(Renv[ri]);
  if (built) dev_sync(dev);  // environment builds are timed as Ren
  stats.t_ren += wall_seconds() - t0;
  build_heff(l);
}

// ------------------------------------------------- interpolative decomposition
// Rows A (m x c, row-major) are approximated as A = T A[skel] with skel a set
// of r rows picked by Gram-Schmidt with pivoting on the largest residual norm
// (a rank-revealing QR of A^T); picking stops once every residual is below
// tol * (largest row norm).  One pass: the projection of each row on each
// new basis vector is recorded as it is removed, which gives the
// coefficients C (m x r) of every row in the orthonormal basis (lower
// triangular on the skeleton rows), and the final residuals are the
// reconstruction errors.  Returns false (no compression) when r is not below m
// or a residual exceeds check * (largest row norm).
static bool interp_decomp(const std::vector<double> &A, int m, int c, double tol, double check,
                          std::vector<int> &skel, std::vector<double> &T) {
  std::vector<double> Rr(A);
  std::vector<double> nrm(m, 0.0);
  double amax = 0.0;
  for (int i = 0; i < m; ++i) {
    double s2 = 0.0;
    for (int j = 0; j < c; ++j) s2 += A[size_t(i) * c + j] * A[size_t(i) * c + j];
    nrm[i] = s2;
    amax = std::max(amax, std::sqrt(s2));
  }
  skel.clear();
  if (amax == 0.0 || m < 2) return false;
  std::vector<std::vector<double>> Q;
  std::vector<std::vector<double>> coef(m);  // coef[i][k] = A_i . q_k
  std::vector<char> used(m, 0);
  for (;;) {
    int best = -1;
    double bn = 0.0;
    for (int i = 0; i < m; ++i)
      if (!used[i] && nrm[i] > bn) {
        bn = nrm[i];
        best = i;
      }
    if (best < 0 || std::sqrt(bn) <= tol * amax) break;
    if (int(skel.size()) + 1 >= m) return false;  // no reduction
    std::vector<double> q(Rr.begin() + size_t(best) * c, Rr.begin() + size_t(best + 1) * c);
    // reorthogonalise the picked residual against the basis (its earlier
    // projections are already in coef[best]; the corrections are added)
    for (size_t k = 0; k < Q.size(); ++k) {
      double d = 0.0;
      for (int j = 0; j < c; ++j) d += Q[k][j] * q[j];
      for (int j = 0; j < c; ++j) q[j] -= d * Q[k][j];
      coef[best][k] += d;
    }
    double qn = 0.0;
    for (double v : q) qn += v * v;
    qn = std::sqrt(qn);
    if (qn <= tol * amax) break;
    for (double &v : q) v /= qn;
    used[best] = 1;
    coef[best].push_back(qn);
    skel.push_back(best);
    for (int i = 0; i < m; ++i) {
      if (used[i]) continue;
      double *ri = &Rr[size_t(i) * c];
      double d = 0.0;
      for (int j = 0; j < c; ++j) d += ri[j] * q[j];
      double s2 = 0.0;
      for (int j = 0; j < c; ++j) {
        ri[j] -= d * q[j];
        s2 += ri[j] * ri[j];
      }
      nrm[i] = s2;
      coef[i].resize(skel.size() - 1, 0.0);
      coef[i].push_back(d);
    }
    Q.push_back(std::move(q));
  }
  const int r = int(skel.size());
  if (r == 0 || r >= m) return false;
  for (int i = 0; i < m; ++i)
    if (!used[i] && std::sqrt(nrm[i]) > check * amax) return false;
  // T C[skel] = C, with C[skel] lower triangular in pick order
  auto C = [&](int i, int k) { return k < int(coef[i].size()) ? coef[i][k] : 0.0; };
  T.assign(size_t(m) * r, 0.0);
  for (int i = 0; i < m; ++i)
    for (int k = r - 1; k >= 0; --k) {
      double v = C(i, k);
      for (int k2 = k + 1; k2 < r; ++k2) v -= T[size_t(i) * r + k2] * C(skel[k2], k);
      T[size_t(i) * r + k] = v / C(skel[k], k);
    }
  return true;
}

// ------------------------------------------------------------- H_eff
void Context::build_heff(int l) {
  double t0 = wall_seconds();
  release_bond();
  last_decimated = 0;
  const Hamiltonian &H = ham;
  const int d = H.d, d2 = d * d;
  const OpSet &L = *Lenv[l];
  const OpSet &R = *Renv[l + 2];
  psi = make_layout(l);
  struct Item {
    std::vector<double> O;
    int parity = 0;
  };
  std::map<std::pair<OpRef, OpRef>, Item> items;
  std::set<std::tuple<OpRef, OpRef, uint64_t, uint64_t>> seen;
  std::set<uint64_t> wantL, wantR;
  auto two_site = [&](const int *e1, int k1, const int *e2, int k2) {
    std::vector<double> X1 = H.site_matrix(l, e1, k1), X2 = H.site_matrix(l + 1, e2, k2);
    std::vector<double> O(d2 * d2, 0.0);
    for (int a1 = 0; a1 < d; ++a1)
      for (int b1 = 0; b1 < d; ++b1) {
        if (X1[a1 * d + b1] == 0.0) continue;
        const double sg = ((k2 & 1) && parity_of_state(b1)) ? -1.0 : 1.0;
        for (int a2 = 0; a2 < d; ++a2)
          for (int b2 = 0; b2 < d; ++b2)
            O[(a1 * d + a2) * d2 + b1 * d + b2] += sg * X1[a1 * d + b1] * X2[a2 * d + b2];
      }
    return O;
  };
  auto add_item2 = [&](OpRef lr, OpRef rr, const std::vector<double> &O, int par, double c) {
    auto &it = items[{lr, rr}];
    if (it.O.empty()) it.O.assign(d2 * d2, 0.0);
    it.parity = par;
    for (int i = 0; i < d2 * d2; ++i) it.O[i] += c * O[i];
  };
  auto add_set = [&](OpRef lr, OpRef rr, const int *e1, int k1, const int *e2, int k2) {
    const auto key = std::make_tuple(lr, rr, make_key(K_N, e1, k1), make_key(K_N, e2, k2));
    if (!seen.insert(key).second) return;
    add_item2(lr, rr, two_site(e1, k1, e2, k2), (k1 + k2) & 1, 1.0);
    if (lr.src == 2) wantL.insert(lr.key);
    if (rr.src == 2) wantR.insert(rr.key);
  };
  const uint64_t kH = make_key(K_H, nullptr, 0);
  const OpRef ident{0, ident_key()};
  {
    std::vector<double> Id(d2 * d2, 0.0);
    for (int i = 0; i < d2; ++i) Id[i * d2 + i] = 1.0;
    add_item2(OpRef{1, kH}, ident, Id, 0, 1.0);
    add_item2(ident, OpRef{1, kH}, Id, 0, 1.0);
  }
  struct CGroup {
    int e1[4] = {}, e2[4] = {}, k1 = 0, k2 = 0, nL = 0;
    QN qL;
    std::vector<uint64_t> rows, rkey, cols;  // left normal key, right complementary key, right string
    std::unordered_map<uint64_t, int> row_of, col_of;
    struct E {
      int r, c;
      double v;
    };
    std::vector<E> entries;
  };
  std::map<std::tuple<uint64_t, int, int64_t>, CGroup> cgroups;  // (site string, ops on site 1, shift of K_L)
  std::map<uint64_t, std::pair<QN, std::map<uint64_t, double>>> zcombos;  // K_Z combos of L
  for (const Term &t : H.terms) {
    Parts p;
    split(H, t, l, p);
    const int kL = p.k[0], kS = p.k[1] + p.k[2], kR = p.k[3];
    if (kL == t.n || kR == t.n) continue;
    if (kL == 0 && kR == 0) {
      add_item2(ident, ident, two_site(p.e[1], p.k[1], p.e[2], p.k[2]), 0, t.c);
      continue;
    }
    if (kR >= 1 && t.n - kR <= 2) {
      int K[4], kk = 0;
      for (int q = 0; q < 3; ++q)
        for (int i = 0; i < p.k[q]; ++i) K[kk++] = p.e[q][i];
      if (compress && kL >= 1) {
        // N^L_{K_L} x O_s x C^R_{K_L s}: collected per (site string s, shift
        // of K_L); the row of K_L holds the coefficients of C^R_{K_L s} over
        // the strings of R, i.e. the coefficients of these terms
        int S[4], ks = 0;
        for (int q = 1; q < 3; ++q)
          for (int i = 0; i < p.k[q]; ++i) S[ks++] = p.e[q][i];
        const QN qL = q_sum(H, p.e[0], kL);
        auto &g = cgroups[std::make_tuple(make_key(K_N, S, ks), p.k[1], qL.key())];
        if (g.rows.empty() && g.cols.empty()) {
          g.k1 = p.k[1];
          g.k2 = p.k[2];
          for (int i = 0; i < p.k[1]; ++i) g.e1[i] = p.e[1][i];
          for (int i = 0; i < p.k[2]; ++i) g.e2[i] = p.e[2][i];
          g.qL = qL;
          g.nL = kL;
        }
        const uint64_t rk = make_key(K_N, p.e[0], kL);
        auto ri = g.row_of.find(rk);
        int row;
        if (ri == g.row_of.end()) {
          row = int(g.rows.size());
          g.row_of[rk] = row;
          g.rows.push_back(rk);
          g.rkey.push_back(make_key(K_C, K, kk));
        } else {
          row = ri->second;
        }
        const uint64_t ck = make_key(K_N, p.e[3], kR);
        auto ci = g.col_of.find(ck);
        int col;
        if (ci == g.col_of.end()) {
          col = int(g.cols.size());
          g.col_of[ck] = col;
          g.cols.push_back(ck);
        } else {
          col = ci->second;
        }
        g.entries.push_back({row, col, t.c});
        continue;
      }
      OpRef lr = kL == 0 ? ident : OpRef{1, make_key(K_N, p.e[0], kL)};
      add_set(lr, OpRef{1, make_key(K_C, K, kk)}, p.e[1], p.k[1], p.e[2], p.k[2]);
      continue;
    }
    if (kR >= 1) {  // kR == 1, three operators outside R
      if (kL == 3) {
        add_set(OpRef{1, make_key(K_C, p.e[3], 1)}, OpRef{1, make_key(K_N, p.e[3], 1)}, nullptr, 0, nullptr, 0);
      } else if (kL == 2) {
        int K[4], kk = 0;
        for (int q = 1; q < 4; ++q)
          for (int i = 0; i < p.k[q]; ++i) K[kk++] = p.e[q][i];
        add_set(OpRef{2, make_key(K_X, K, kk)}, OpRef{1, make_key(K_N, p.e[3], 1)}, p.e[1], p.k[1], p.e[2],
                p.k[2]);
      } else {
        int K[4], kk = 0;
        for (int q = 0; q < 3; ++q)
          for (int i = 0; i < p.k[q]; ++i) K[kk++] = p.e[q][i];
        OpRef lr = kL == 0 ? ident : OpRef{1, make_key(K_N, p.e[0], kL)};
        add_set(lr, OpRef{2, make_key(K_X, K, kk)}, p.e[1], p.k[1], p.e[2], p.k[2]);
      }
      continue;
    }
    // kR == 0, kL >= 1, kS >= 1
    int K[4], kk = 0;
    for (int q = 1; q < 3; ++q)
      for (int i = 0; i < p.k[q]; ++i) K[kk++] = p.e[q][i];
    const bool stored = (t.n == 4 && kL == 3);
    add_set(OpRef{stored ? 1 : 2, make_key(stored ? K_C : K_X, K, kk)}, ident, p.e[1], p.k[1], p.e[2], p.k[2]);
    (void)kS;
  }
  // interpolative compression of each group: sum_K N^L_K x O_s x C^R_{K s}
  // = sum_{j in skel} (sum_K T_Kj N^L_K) x O_s x C^R_{K_j s}, exact because the
  // stored C^R are linear in their coefficients
  int64_t n_before = 0, n_after = 0;
  {
    // decompositions of the groups are independent: host threads take them
    // in turn; the products are then emitted in group order
    std::vector<CGroup *> gl;
    for (auto &gk : cgroups) gl.push_back(&gk.second);
    struct IdOut {
      bool ok = false;
      std::vector<int> skel;
      std::vector<double> T;
    };
    std::vector<IdOut> res(gl.size());
    std::atomic<size_t> next{0};
    auto work = [&] {
      for (size_t gi; (gi = next.fetch_add(1)) < gl.size();) {
        const CGroup &g = *gl[gi];
        const int m = int(g.rows.size()), c = int(g.cols.size());
        std::vector<double> A(size_t(m) * c, 0.0);
        for (auto &e : g.entries) A[size_t(e.r) * c + e.c] += e.v;
        res[gi].ok = m > 1 && interp_decomp(A, m, c, 1e-14, 1e-12, res[gi].skel, res[gi].T);
      }
    };
    const int nth = int(std::min<size_t>(gl.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency()))));
    std::vector<std::thread> pool;
    for (int t = 1; t < nth; ++t) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
    for (size_t gi = 0; gi < gl.size(); ++gi) {
      CGroup &g = *gl[gi];
      const int m = int(g.rows.size());
      n_before += m;
      if (!res[gi].ok) {
        for (int i = 0; i < m; ++i) add_set(OpRef{1, g.rows[i]}, OpRef{1, g.rkey[i]}, g.e1, g.k1, g.e2, g.k2);
        n_after += m;
        continue;
      }
      const std::vector<int> &skel = res[gi].skel;
      const std::vector<double> &T = res[gi].T;
      const int r = int(skel.size());
      n_after += r;
      const std::vector<double> O = two_site(g.e1, g.k1, g.e2, g.k2);
      for (int k = 0; k < r; ++k) {
        const uint64_t zk = uint64_t(K_Z) | (uint64_t(g.nL) << 4) | (uint64_t(zcombos.size()) << 8);
        auto &zc = zcombos[zk];
        zc.first = g.qL;
        for (int i = 0; i < m; ++i) {
          const double v = T[size_t(i) * r + k];
          if (v != 0.0) zc.second[g.rows[i]] += v;
        }
        add_item2(OpRef{2, zk}, OpRef{1, g.rkey[skel[k]]}, O, (g.k1 + g.k2) & 1, 1.0);
      }
    }
  }
  const bool verbose = std::getenv("MDMRG_VERBOSE") != nullptr;
  if (verbose && n_before)
    fprintf(stderr, "[mdmrg] bond %d: N^L x C^R products %lld -> %lld after interpolative compression\n", l,
            (long long)n_before, (long long)n_after);
  double tv[5] = {wall_seconds(), 0, 0, 0, 0};  // verbose sub-timing: products, combos, tasks, plan
  // on-the-fly complementary operators
  if (!wantL.empty() || !zcombos.empty()) {
    Lx = std::make_unique<OpSet>();
    Lx->bond = L.bond;
    for (uint64_t k : wantL) Lx->add(k, combo_delta(H, true, k));
    for (auto &z : zcombos) Lx->add(z.first, z.second.first);
    Lx->layout(dev);
    Content c;
    combo_content(H, true, l, wantL, c);
    for (auto &z : zcombos) c[z.first] = z.second.second;
    materialize(dev, *Lx, L, c);
  }
  if (!wantR.empty()) {
    Rx = std::make_unique<OpSet>();
    Rx->bond = R.bond;
    for (uint64_t k : wantR) Rx->add(k, combo_delta(H, false, k));
    Rx->layout(dev);
    Content c;
    combo_content(H, false, l + 2, wantR, c);
    materialize(dev, *Rx, R, c);
  }
  if (verbose) {
    dev_sync(dev);
    tv[1] = wall_seconds();
  }
  // GEMM tasks
  const Bond &ba = bonds[l], &bb = bonds[l + 2];
  std::vector<PairTask> tasks;
  std::vector<OutBlk> outs(psi.blk.size());
  for (size_t i = 0; i < psi.blk.size(); ++i) {
    const PsiBlk &pb = psi.blk[i];
    outs[i] = OutBlk{1, pb.off, pb.m, pb.n, pb.n};
  }
  std::vector<DiagTask> dtasks;
  heff_terms = int64_t(items.size());
  for (auto &kv : items) {
    const OpRef &lr = kv.first.first, &rr = kv.first.second;
    const Item &it = kv.second;
    const OpSet *Ls = lr.src == 1 ? &L : lr.src == 2 ? Lx.get() : nullptr;
    const OpSet *Rs = rr.src == 1 ? &R : rr.src == 2 ? Rx.get() : nullptr;
    if ((lr.src && !Ls->has(lr.key)) || (rr.src && !Rs->has(rr.key))) continue;  // zero operator
    const int pR = rr.src ? key_parity(rr.key) : 0;
    const int pS = it.parity;
    for (const PsiBlk &pb : psi.blk) {
      // L block a -> a'
      int ap = pb.a, bp = pb.b;
      int64_t loff = -1, roff = -1;
      if (lr.src) {
        loff = Ls->block(lr.key, pb.a, &ap);
        if (loff < 0) continue;
      }
      if (rr.src) {
        roff = Rs->block(rr.key, pb.b, &bp);
        if (roff < 0) continue;
      }
      const int pa = ba.qn[pb.a].parity();
      const int col = pb.s1 * d + pb.s2;
      for (int s1p = 0; s1p < d; ++s1p)
        for (int s2p = 0; s2p < d; ++s2p) {
          const double o = it.O[(s1p * d + s2p) * d2 + col];
          if (o == 0.0) continue;
          const int oi = psi.find(ap, s1p, s2p, bp);
          if (oi < 0) continue;
          const int ex = pR * (pa + parity_of_state(pb.s1) + parity_of_state(pb.s2)) + pS * pa;
          const double alpha = o * ((ex & 1) ? -1.0 : 1.0);
          PairTask t{};
          t.out = oi;
          t.m = ba.dim[ap];
          t.k1 = pb.m;
          t.k2 = pb.n;
          t.n = bb.dim[bp];
          t.alpha = alpha;
          t.X = Ref{0, pb.off, pb.n};
          if (lr.src)
            t.A = Ref{lr.src == 1 ? 3 : 5, loff, pb.m};
          else
            t.idA = true;
          if (rr.src) {
            t.B = Ref{rr.src == 1 ? 4 : 6, roff, pb.n};
            t.tB = true;
          } else {
            t.idB = true;
          }
          tasks.push_back(t);
          // diagonal contribution
          if (oi == int(&pb - &psi.blk[0]) && ap == pb.a && bp == pb.b) {
            DiagTask dt{};
            dt.d_off = pb.off;
            dt.alpha = alpha;
            dt.m = pb.m;
            dt.n = pb.n;
            dt.l_id = lr.src ? 0 : 1;
            dt.r_id = rr.src ? 0 : 1;
            dt.l_slot = uint8_t(lr.src == 1 ? 3 : 5);
            dt.r_slot = uint8_t(rr.src == 1 ? 4 : 6);
            dt.l_off = loff;
            dt.r_off = roff;
            dt.ls = pb.m + 1;
            dt.rs = pb.n + 1;
            dtasks.push_back(dt);
          }
        }
    }
  }
  if (std::getenv("MDMRG_VERBOSE")) {
    // flop-weighted histogram of the largest GEMM dimension
    const int edges[] = {8, 16, 32, 64, 128, 256, 512, 1 << 30};
    double hist[8] = {0};
    for (const PairTask &t : tasks) {
      const int mx = std::max(std::max(t.m, t.n), std::max(t.k1, t.k2));
      int bin = 0;
      while (mx > edges[bin]) ++bin;
      hist[bin] += 2.0 * t.m * t.k1 * t.k2 + 2.0 * t.m * t.k2 * t.n;
    }
    double tot = 0;
    for (double h : hist) tot += h;
    fprintf(stderr, "[mdmrg] bond %d: psi %lld elems in %zu blocks, %zu products, %zu pair tasks; flop share by max dim",
            l, (long long)psi.n_elem, psi.blk.size(), items.size(), tasks.size());
    for (int i = 0; i < 8; ++i) fprintf(stderr, " <=%d:%.2f", edges[i], tot > 0 ? hist[i] / tot : 0.0);
    fprintf(stderr, "\n");
  }
  if (verbose) tv[2] = wall_seconds();
  build_two_phase(tasks, outs, scratch_limit, heff, dev, psi.n_elem);
  if (verbose) tv[3] = wall_seconds();
  if (heff.n_split > 1 && P_scratch_n < heff.n_split * psi.n_elem) {
    release_graphs();
    if (P_scratch) dev_free(dev, P_scratch);
    P_scratch_n = heff.n_split * psi.n_elem;
    P_scratch = (double *)dev_alloc(dev, sizeof(double) * P_scratch_n);
  }
  if (std::getenv("MDMRG_VERBOSE")) {
    int64_t tiles = 0, s1 = 0, s2 = 0, o2 = 0;
    for (auto &c : heff.chunks) {
      for (DevPlan *p : {c.p1, c.p2})
        if (p) tiles += p->n_tiles;
      if (c.p1) s1 += c.p1->n_segs;
      if (c.p2) {
        s2 += c.p2->n_segs;
        o2 += c.p2->n_outs;
      }
    }
    fprintf(stderr,
            "[mdmrg] bond %d: %zu chunks, scratch %.2f GB, flop %.3e, bytes %.3e, phase-1 outputs %lld, phase-2 "
            "outputs %lld with %lld segments (split-K %d), tiles %lld\n",
            l, heff.chunks.size(), heff.scratch * 8e-9, heff.flop, heff.bytes, (long long)s1, (long long)o2,
            (long long)s2, heff.n_split, (long long)tiles);
  }
  ensure_scratch(heff.scratch);
  std::vector<int64_t> boff;
  std::vector<int32_t> bm, bn;
  for (auto &pb : psi.blk) {
    boff.push_back(pb.off);
    bm.push_back(pb.m);
    bn.push_back(pb.n);
  }
  diag = dev_diag_upload(dev, dtasks, boff, bm, bn);
  cur = l;
  dev_sync(dev);
  if (verbose)
    fprintf(stderr, "[mdmrg] bond %d tables: products %.3fs, combos %.3fs, tasks %.3fs, plan %.3fs, rest %.3fs\n", l,
            tv[0] - t0, tv[1] - tv[0], tv[2] - tv[1], tv[3] - tv[2], wall_seconds() - tv[3]);
  stats.t_tables += wall_seconds() - t0;
}

void Context::ensure_fp32() {
  if (x32) return;
  auto shadow = [&](const OpSet *S) -> float * {
    if (!S || !S->arena) return nullptr;
    float *f = (float *)dev_alloc(dev, sizeof(float) * std::max<int64_t>(1, S->arena_size));
    dev_d2f(dev, S->arena, f, S->arena_size);
    return f;
  };
  L32 = shadow(Lenv[cur].get());
  R32 = shadow(Renv[cur + 2].get());
  Lx32 = shadow(Lx.get());
  Rx32 = shadow(Rx.get());
  x32 = (float *)dev_alloc(dev, sizeof(float) * std::max<int64_t>(1, psi.n_elem));
  y32 = (float *)dev_alloc(dev, sizeof(float) * std::max<int64_t>(1, psi.n_elem));
}

void Context::heff_apply(const double *x, double *y, int prec) {
  MDMRG_REQUIRE(cur >= 0, -4, "heff_apply: no current bond");
  MDMRG_REQUIRE(prec >= 0 && prec < kPrecs, -6, "heff_apply: unknown precision form");
  // a graph is captured once every plan of the product has finished its
  // variant trials (kGemmVariants timed launches, decided at the next one)
  const int warm = kGemmVariants + 1;
  if (prec != 0) {
    // split forms: FP32 shadows of x, y and the operators; prec 1 runs FP32
    // MFMA products, prec 2 the 3xBF16 and prec 3 the 6xBF16 products on
    // the same data
    DevGraph *&graph = prec == 1 ? graph32 : prec == 2 ? graphbf3 : graphbf6;
    int &eager = prec == 1 ? eager32 : prec == 2 ? eagerbf3 : eagerbf6;
    ensure_fp32();
    dev_d2f(dev, x, x32, psi.n_elem);
    Bases b{};
    b.p[0] = reinterpret_cast<double *>(x32);
    b.p[1] = reinterpret_cast<double *>(y32);
    b.p[3] = reinterpret_cast<double *>(L32);
    b.p[4] = reinterpret_cast<double *>(R32);
    b.p[5] = Lx32 ? reinterpret_cast<double *>(Lx32) : b.p[3];
    b.p[6] = Rx32 ? reinterpret_cast<double *>(Rx32) : b.p[4];
    b.p[7] = b.p[1];
    auto body = [&] {
      dev_zero(dev, y32, sizeof(float) * psi.n_elem);
      run_plan(heff, b, 4, prec);
    };
    if (use_graph && !graph && eager >= warm) {
      dev_capture_begin(dev);
      try {
        body();
      } catch (...) {
        dev_capture_abort(dev);
        throw;
      }
      graph = dev_capture_end(dev);
    }
    if (graph) {
      dev_graph_launch(dev, graph, 7 + prec, heff.flop);
    } else {
      body();
      ++eager;
    }
    dev_f2d(dev, y32, y, psi.n_elem);
    stats.heff_flop_split += heff.flop;
    stats.n_matvec_split += 1;
    return;
  }
  Bases b{};
  b.p[3] = Lenv[cur]->arena;
  b.p[4] = Renv[cur + 2]->arena;
  b.p[5] = Lx ? Lx->arena : b.p[3];
  b.p[6] = Rx ? Rx->arena : b.p[4];
  if (use_graph && eager64 >= warm) {
    if (!graph64) {
      if (xg_n < psi.n_elem) {
        for (double **p : {&xg, &yg}) {
          if (*p) dev_free(dev, *p);
          *p = (double *)dev_alloc(dev, sizeof(double) * psi.n_elem);
        }
        xg_n = psi.n_elem;
      }
      b.p[0] = xg;
      b.p[1] = yg;
      b.p[7] = yg;
      dev_capture_begin(dev);
      try {
        dev_zero(dev, yg, sizeof(double) * psi.n_elem);
        run_plan(heff, b, 1);
      } catch (...) {
        dev_capture_abort(dev);
        throw;
      }
      graph64 = dev_capture_end(dev);
    }
    dev_d2d(dev, xg, x, sizeof(double) * psi.n_elem);
    dev_graph_launch(dev, graph64, 7, heff.flop);
    dev_d2d(dev, y, yg, sizeof(double) * psi.n_elem);
  } else {
    b.p[0] = const_cast<double *>(x);
    b.p[1] = y;
    b.p[7] = y;
    dev_zero(dev, y, sizeof(double) * psi.n_elem);
    run_plan(heff, b, 1);
    ++eager64;
  }
  stats.heff_flop += heff.flop;
  stats.n_matvec += 1;
}

void Context::heff_diag(double *dd) {
  MDMRG_REQUIRE(cur >= 0, -4, "heff_diag: no current bond");
  dev_zero(dev, dd, sizeof(double) * psi.n_elem);
  Bases b{};
  b.p[0] = dd;
  b.p[1] = dd;
  b.p[2] = dd;
  b.p[3] = Lenv[cur]->arena;
  b.p[4] = Renv[cur + 2]->arena;
  b.p[5] = Lx ? Lx->arena : b.p[3];
  b.p[6] = Rx ? Rx->arena : b.p[4];
  b.p[7] = dd;
  dev_diag_run(dev, diag, b, dd);
}

// ------------------------------------------------------------- Davidson
// cyclic Jacobi eigen-decomposition of a small symmetric matrix (row-major)
static void jacobi_eig(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> &V) {
  V.assign(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          const double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return A[a * n + a] < A[b * n + b]; });
  w.resize(n);
  std::vector<double> V2(size_t(n) * n);
  for (int j = 0; j < n; ++j) {
    w[j] = A[idx[j] * n + idx[j]];
    for (int k = 0; k < n; ++k) V2[k * n + j] = V[k * n + idx[j]];
  }
  V = V2;
}

// One product of a Davidson solve: H_eff v in form prec, plus, for a split
// form while a defect correction is set (davidson_mixed), the symmetric
// rank-2 term C v = d (x0.v) + x0 (d.v) - gamma x0 (x0.v).  Since
// d = H x0 - H_split x0 is the FP64 defect of the split operator at the
// normalised vector x0, the corrected operator reproduces H x0 exactly and
// differs from H, near x0, only by the split rounding of the difference
// (first order in |x - x0|).
void Context::davidson_product(const double *v, double *w, int prec) {
  heff_apply(v, w, prec);
  if (corr && prec != 0) {
    const int64_t N = psi.n_elem;
    double ab[2];  // x0.v, d.v
    dev_multidot(dev, corr, N, 2, v, N, ab);
    const double c[2] = {ab[1] - corr_gamma * ab[0], ab[0]};
    dev_lincomb(dev, corr, N, 2, c, 1.0, w, N);
  }
}

int Context::davidson(double *x, double tol, int max_iter, int m_max, double *energy, double *resid,
                      int *n_mv, int prec, double stall_floor, const double *V0, int k0, double *Vout, int kout,
                      int *k_written, const double *hx_start) {
  MDMRG_REQUIRE(cur >= 0, -4, "davidson: no current bond");
  MDMRG_REQUIRE(m_max >= 3 && m_max <= 60, -1, "davidson: m_max must be in [3, 60]");
  const bool verbose = std::getenv("MDMRG_VERBOSE") != nullptr;
  const int64_t N = psi.n_elem;
  double t0 = wall_seconds();
  DevVecs work(dev);
  double *V = work.get(N * m_max);
  double *AV = work.get(N * m_max);
  double *dg = work.get(N);
  double *r = work.get(N);
  double *ax = work.get(N);
  double *px = davidson_olsen ? work.get(N) : nullptr;
  heff_diag(dg);
  // start vector
  double nrm;
  dev_multidot(dev, x, 0, 1, x, N, &nrm);
  // a non-finite start vector is an error (checked before the zero test,
  // which a NaN norm would also fail); only an exact zero is replaced
  MDMRG_REQUIRE(std::isfinite(nrm), -3, "davidson: start vector is not finite");
  if (!(nrm > 1e-300)) {
    dev_randn(dev, x, N, 3);
    dev_multidot(dev, x, 0, 1, x, N, &nrm);
  }
  dev_d2d(dev, V, x, sizeof(double) * N);
  dev_scale(dev, 1.0 / std::sqrt(nrm), V, N);
  // hx_start: the product of the (normalised) start vector, already formed
  // by the caller in this form and counted there
  if (hx_start)
    dev_d2d(dev, AV, hx_start, sizeof(double) * N);
  else
    davidson_product(V, AV, prec);
  int nmv = hx_start ? 0 : 1, nv = 1;
  double best_r = 1e300;
  int best_at = 0;
  floor_checks = 0;
  std::vector<double> Hs(size_t(m_max) * m_max, 0.0);
  {
    double h;
    dev_multidot(dev, V, 0, 1, AV, N, &h);
    Hs[0] = h;
  }
  // further start vectors (Ritz vectors of an earlier solve in another
  // precision): orthonormalised against the subspace, one product each
  for (int j = 1; j < k0 && nv < m_max - 2; ++j) {
    double *t = V + int64_t(nv) * N;
    dev_d2d(dev, t, V0 + int64_t(j) * N, sizeof(double) * N);
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<double> c(nv);
      dev_multidot(dev, V, N, nv, t, N, c.data());
      for (auto &v : c) v = -v;
      dev_lincomb(dev, V, N, nv, c.data(), 1.0, t, N);
    }
    double tn;
    dev_multidot(dev, t, 0, 1, t, N, &tn);
    if (!(tn > 1e-20)) continue;
    dev_scale(dev, 1.0 / std::sqrt(tn), t, N);
    davidson_product(t, AV + int64_t(nv) * N, prec);
    ++nmv;
    std::vector<double> col(nv + 1);
    dev_multidot(dev, V, N, nv + 1, AV + int64_t(nv) * N, N, col.data());
    for (int i = 0; i <= nv; ++i) {
      Hs[i * m_max + nv] = col[i];
      Hs[nv * m_max + i] = col[i];
    }
    ++nv;
  }
  double theta = Hs[0], rn = 1e300;
  int status = 0;
  std::vector<double> w, Y;
  int nv_y = 0;  // subspace size of the Ritz vectors in Y
  while (true) {
    std::vector<double> S(size_t(nv) * nv);
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < nv; ++j) S[i * nv + j] = 0.5 * (Hs[i * m_max + j] + Hs[j * m_max + i]);
    jacobi_eig(nv, S, w, Y);
    nv_y = nv;
    theta = w[0];
    std::vector<double> y(nv);
    for (int i = 0; i < nv; ++i) y[i] = Y[i * nv + 0];
    dev_lincomb(dev, V, N, nv, y.data(), 0.0, x, N);
    dev_lincomb(dev, AV, N, nv, y.data(), 0.0, ax, N);
    dev_d2d(dev, r, ax, sizeof(double) * N);
    dev_axpy(dev, -theta, x, r, N);
    double r2;
    dev_multidot(dev, r, 0, 1, r, N, &r2);
    MDMRG_REQUIRE(std::isfinite(r2) && std::isfinite(theta), -3, "davidson: NaN in residual");
    rn = std::sqrt(r2);
    if (verbose) fprintf(stderr, "[mdmrg] davidson: %d products, |r| = %.3e\n", nmv, rn);
    if (rn <= tol) break;
    if (nmv >= max_iter) {
      status = -5;
      break;
    }
    if (stall_floor >= 0.0) {
      // the split-precision operator has a noise floor: stop once the
      // residual has not dropped by 10% over the last 4 products within
      // twice the measured floor, over 24 within 20 times it, and over 64
      // elsewhere (far above the floor a plateau is slow convergence, e.g.
      // after a restart, not the floor)
      // (a defect-corrected stage stops after 8 products without a 10% gain,
      // without floor checks: a new defect round re-centres the correction)
      const int window = corr ? 8 : rn <= 2.0 * stall_floor ? 4 : rn <= 20.0 * stall_floor ? 24 : 64;
      if (rn < 0.9 * best_r) {
        best_r = rn;
        best_at = nmv;
      } else if (nmv - best_at >= window) {
        if (corr) break;
        // the floor, or slow convergence (a plateau after a restart)?  One
        // FP64 product of the Ritz vector decides: an FP64 residual close to
        // the split one means the split operator's rounding is not what
        // stops progress, so the split solve goes on (at most 3 checks)
        if (prec == 0 || floor_checks >= 3) break;
        DevVecs tmp(dev);
        double *hx = tmp.get(N);
        heff_apply(x, hx, 0);
        ++floor_checks;
        double xh = 0.0, r2 = 0.0;
        dev_multidot(dev, x, 0, 1, hx, N, &xh);
        dev_axpy(dev, -xh, x, hx, N);  // FP64 residual H x - (x.Hx) x, |x| = 1
        dev_multidot(dev, hx, 0, 1, hx, N, &r2);
        const double r64 = std::sqrt(r2);
        if (verbose) fprintf(stderr, "[mdmrg] davidson: split |r| = %.3e, FP64 |r| = %.3e\n", rn, r64);
        if (!(r64 <= 2.0 * rn)) break;
        best_r = rn;
        best_at = nmv;
      }
    }
    if (nv == m_max) {
      // thick restart to the lowest Ritz vectors (x first): their products
      // follow from the stored ones, so the restart costs no product
      const int keep = std::max(2, std::min(davidson_keep, m_max - 2));
      DevVecs tmp(dev);
      double *tv = tmp.get(int64_t(keep) * N), *tav = tmp.get(int64_t(keep) * N);
      std::vector<double> yk(nv);
      for (int c = 0; c < keep; ++c) {
        for (int i = 0; i < nv; ++i) yk[i] = Y[i * nv + c];
        dev_lincomb(dev, V, N, nv, yk.data(), 0.0, tv + int64_t(c) * N, N);
        dev_lincomb(dev, AV, N, nv, yk.data(), 0.0, tav + int64_t(c) * N, N);
      }
      dev_d2d(dev, V, tv, sizeof(double) * N * keep);
      dev_d2d(dev, AV, tav, sizeof(double) * N * keep);
      std::fill(Hs.begin(), Hs.end(), 0.0);
      std::vector<double> h(keep);
      for (int j = 0; j < keep; ++j) {
        dev_multidot(dev, V, N, keep, AV + int64_t(j) * N, N, h.data());
        for (int i = 0; i < keep; ++i) Hs[i * m_max + j] = h[i];
      }
      nv = keep;
      // residual of x (the first kept vector)
      dev_d2d(dev, r, ax, sizeof(double) * N);
      dev_axpy(dev, -theta, x, r, N);
    }
    // correction vector: t = P r with P = (theta - diag H)^-1 (Davidson);
    // with the Olsen variant t = P r - eps P x, eps = (x.P r)/(x.P x), which
    // removes the component of the correction that merely rescales x
    double *t = V + int64_t(nv) * N;
    dev_precond(dev, r, dg, theta, 1e-8, t, N);
    if (davidson_olsen) {
      dev_precond(dev, x, dg, theta, 1e-8, px, N);
      double xt = 0.0, xp = 0.0;
      dev_multidot(dev, x, 0, 1, t, N, &xt);
      dev_multidot(dev, x, 0, 1, px, N, &xp);
      if (std::fabs(xp) > 1e-300) dev_axpy(dev, -xt / xp, px, t, N);
    }
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<double> c(nv);
      dev_multidot(dev, V, N, nv, t, N, c.data());
      for (auto &v : c) v = -v;
      dev_lincomb(dev, V, N, nv, c.data(), 1.0, t, N);
    }
    double tn;
    dev_multidot(dev, t, 0, 1, t, N, &tn);
    if (!(tn > 1e-28)) {
      // preconditioned residual collapsed into the subspace: use r itself
      dev_d2d(dev, t, r, sizeof(double) * N);
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<double> c(nv);
        dev_multidot(dev, V, N, nv, t, N, c.data());
        for (auto &v : c) v = -v;
        dev_lincomb(dev, V, N, nv, c.data(), 1.0, t, N);
      }
      dev_multidot(dev, t, 0, 1, t, N, &tn);
      if (!(tn > 1e-28)) {
        // no new direction: the subspace is exhausted before tol was reached
        status = -5;
        break;
      }
    }
    dev_scale(dev, 1.0 / std::sqrt(tn), t, N);
    davidson_product(t, AV + int64_t(nv) * N, prec);
    ++nmv;
    std::vector<double> col(nv + 1);
    dev_multidot(dev, V, N, nv + 1, AV + int64_t(nv) * N, N, col.data());
    for (int i = 0; i <= nv; ++i) {
      Hs[i * m_max + nv] = col[i];
      Hs[nv * m_max + i] = col[i];
    }
    ++nv;
  }
  // the lowest Ritz vectors of the final subspace, for a following solve
  if (k_written) *k_written = 0;
  if (Vout && kout > 0 && !Y.empty() && nv_y == nv) {
    const int kk = std::min(kout, nv);
    std::vector<double> yk(nv);
    for (int c = 0; c < kk; ++c) {
      for (int i = 0; i < nv; ++i) yk[i] = Y[i * nv + c];
      dev_lincomb(dev, V, N, nv, yk.data(), 0.0, Vout + int64_t(c) * N, N);
    }
    if (k_written) *k_written = kk;
  }
  // normalise the returned vector
  double xn;
  dev_multidot(dev, x, 0, 1, x, N, &xn);
  dev_scale(dev, 1.0 / std::sqrt(xn), x, N);
  dev_sync(dev);
  if (energy) *energy = theta;
  if (resid) *resid = rn;
  if (n_mv) *n_mv = nmv;
  stats.t_diag_h += wall_seconds() - t0;
  return status;
}

int Context::davidson_mixed(double *x, double tol, int prec_split, double tol_split, int max_iter, int m_max,
                            double *energy, double *resid, int *n_mv64, int *n_mv_split) {
  MDMRG_REQUIRE(prec_split >= 1 && prec_split < kPrecs, -6, "davidson_mixed: prec_split must be a split form");
  MDMRG_REQUIRE(cur >= 0, -4, "davidson_mixed: no current bond");
  // Noise floor of the split operator at this bond, from one split and one
  // FP64 product of the normalised start vector v: the relative
  // perturbation |(H_split - H) v| / |H v| times the Rayleigh quotient
  // |v.Hv| (the scale of |H x| near the eigenvector; |H v| of a random start
  // is larger).  The split solve runs to tol_split or until its residual
  // stagnates; within twice the floor it stops after 4 products without a
  // 10% gain (24 elsewhere), since there split iterations do little for the
  // FP64 residual.
  double floor = 0.0, floor32 = 0.0;
  int probe = 0;
  {
    const int64_t N = psi.n_elem;
    double nrm = 0.0;
    dev_multidot(dev, x, 0, 1, x, N, &nrm);
    if (nrm > 1e-300 && std::isfinite(nrm)) {
      DevVecs work(dev);
      double *v = work.get(N), *a = work.get(N), *b = work.get(N);
      dev_d2d(dev, v, x, sizeof(double) * N);
      dev_scale(dev, 1.0 / std::sqrt(nrm), v, N);
      heff_apply(v, a, prec_split);
      heff_apply(v, b, 0);
      dev_axpy(dev, -1.0, b, a, N);
      double d2 = 0.0, h2 = 0.0, th = 0.0;
      dev_multidot(dev, a, 0, 1, a, N, &d2);
      dev_multidot(dev, b, 0, 1, b, N, &h2);
      dev_multidot(dev, v, 0, 1, b, N, &th);
      if (h2 > 0.0 && std::isfinite(d2)) floor = std::sqrt(d2 / h2) * std::fabs(th);
      if (prec_split == 2 && mixed_ladder) {
        // floor of the FP32 stage from one FP32 product of the same vector
        heff_apply(v, a, 1);
        dev_axpy(dev, -1.0, b, a, N);
        dev_multidot(dev, a, 0, 1, a, N, &d2);
        if (h2 > 0.0 && std::isfinite(d2)) floor32 = std::max(1e-300, std::sqrt(d2 / h2) * std::fabs(th));
      }
      probe = 1;
    }
  }
  double e = 0.0, r = 0.0;
  int ns = 0, n64 = 0;
  const bool verbose = std::getenv("MDMRG_VERBOSE") != nullptr;
  // the next stage starts from the lowest Ritz vectors of the previous one
  // (MDMRG_OPT_MIXED_HANDOVER; 1 = the eigenvector estimate alone), one
  // product each in its own precision
  const int kh = std::max(1, std::min(mixed_handover, m_max - 3));
  DevVecs hand(dev);
  double *Vk = kh > 1 ? hand.get(int64_t(kh) * psi.n_elem) : nullptr;
  int kw = 0;
  davidson(x, std::max(tol, tol_split), max_iter, m_max, &e, &r, &ns, prec_split, floor, nullptr, 0, Vk, kh, &kw);
  int checks = floor_checks;  // FP64 products of the split stages' floor checks
  if (verbose)
    fprintf(stderr, "[mdmrg] mixed: split stage %d products, |r| = %.3e (floor %.3e)\n", ns, r, floor);
  if (prec_split == 2 && mixed_ladder) {
    // FP32 stage between the 3xBF16 and the FP64 solves: it takes the
    // residual from the 3xBF16 floor down towards tol_split at FP32 cost
    int n32 = 0;
    davidson(x, std::max(tol, tol_split), max_iter, m_max, &e, &r, &n32, 1, floor32, Vk, kw, Vk, kh, &kw);
    ns += n32;
    checks += floor_checks;
    if (verbose)
      fprintf(stderr, "[mdmrg] mixed: FP32 stage %d products, |r| = %.3e (floor %.3e)\n", n32, r, floor32);
  }
  // Defect correction (MDMRG_OPT_MIXED_CORRECT): one FP64 product of the
  // current vector x0 gives its FP64 residual (done if within tol, with the
  // FP64 Rayleigh quotient as the energy) and, with one split product, the
  // defect d = H x0 - H_split x0.  A split stage on H_split + C (C the
  // symmetric rank-2 term of davidson_product, so that (H_split + C) x0 =
  // H x0) then carries the residual below the split form's own noise
  // floor: what remains of the rounding acts on x - x0 only.  A corrected
  // stage that stalls (8 products without a 10% gain) ends its round; the
  // next round re-centres the correction at the new vector.  Four rounds at
  // most; once the FP64 residual is within 4 tol the plain FP64 stage
  // finishes from the vector and its FP64 product.
  int n64c = 0, nc = 0, st64 = 0;
  bool done = false;
  if (mixed_correct) {
    const int64_t N = psi.n_elem;
    DevVecs cw(dev);
    double *xd = cw.get(2 * N), *hs = cw.get(N);
    struct Reset {
      const double *&p;
      ~Reset() { p = nullptr; }
    } reset{corr};
    for (int round = 0;; ++round) {
      dev_d2d(dev, xd, x, sizeof(double) * N);  // x is normalised by davidson()
      heff_apply(xd, xd + N, 0);
      ++n64c;
      double th = 0.0, r2 = 0.0;
      dev_multidot(dev, xd, 0, 1, xd + N, N, &th);
      dev_d2d(dev, hs, xd + N, sizeof(double) * N);
      dev_axpy(dev, -th, xd, hs, N);
      dev_multidot(dev, hs, 0, 1, hs, N, &r2);
      MDMRG_REQUIRE(std::isfinite(r2) && std::isfinite(th), -3, "davidson_mixed: NaN in residual");
      const double r64 = std::sqrt(r2);
      if (verbose) fprintf(stderr, "[mdmrg] mixed: FP64 residual %.3e at round %d\n", r64, round);
      if (r64 <= tol) {
        e = th;
        r = r64;
        done = true;
        break;
      }
      if (round == 4 || r64 <= 4.0 * tol) {
        // close to tol (or two rounds spent): the FP64 stage, from this
        // vector and its FP64 product
        st64 = davidson(x, tol, max_iter, m_max, &e, &r, &n64, 0, -1.0, nullptr, 0, nullptr, 0, nullptr, xd + N);
        done = true;
        break;
      }
      heff_apply(xd, hs, prec_split);
      ++nc;
      dev_axpy(dev, -1.0, hs, xd + N, N);  // d = H x0 - H_split x0
      dev_multidot(dev, xd, 0, 1, xd + N, N, &corr_gamma);
      corr = xd;
      int nci = 0;
      davidson(x, 0.5 * tol, max_iter, m_max, &e, &r, &nci, prec_split, 0.5 * tol);
      corr = nullptr;
      nc += nci;
      checks += floor_checks;
      if (verbose) fprintf(stderr, "[mdmrg] mixed: corrected stage %d products, |r| = %.3e\n", nci, r);
    }
  }
  const int st = done ? st64 : davidson(x, tol, max_iter, m_max, &e, &r, &n64, 0, -1.0, Vk, kw);
  ns += probe + (floor32 > 0.0 ? 1 : 0) + nc;
  n64 += probe + checks + n64c;
  if (energy) *energy = e;
  if (resid) *resid = r;
  if (n_mv64) *n_mv64 = n64;
  if (n_mv_split) *n_mv_split = ns;
  return st;
}

// ------------------------------------------------------------- decimation
void Context::decimate(const double *x, int D, int dir, double *trunc, double *svn, double *shalf) {
  MDMRG_REQUIRE(cur >= 0, -4, "decimate: no current bond");
  MDMRG_REQUIRE(D >= 1, -1, "decimate: D must be positive");
  MDMRG_REQUIRE(dir == 1 || dir == -1, -1, "decimate: direction must be +1 or -1");
  double t0 = wall_seconds();
  const int l = cur, d = ham.d;
  const Bond &ba = bonds[l], &bb = bonds[l + 2];
  // |x|^2 = tr(x x^T): refuse a zero or non-finite vector before any
  // eigensolver sees it; rho is formed from x / |x| (trace 1), so that the
  // eigensolver sees the same matrix for any scale of x
  double nx = 0.0;
  dev_multidot(dev, x, 0, 1, x, psi.n_elem, &nx);
  MDMRG_REQUIRE(std::isfinite(nx), -3, "decimate: x is not finite");
  MDMRG_REQUIRE(nx > 0.0, -1, "decimate: zero vector");
  const double rho_scale = 1.0 / nx;
  // enlarged-block sectors and their row lists
  struct Sec {
    QN q;
    std::vector<std::pair<int, int>> rows;  // (sector, local state) for dir +1 : (a,s1); dir -1: (s2,b)
    std::vector<int> roff;
    int M = 0;
    int64_t base = 0;
  };
  std::map<int64_t, int> sidx;
  std::vector<Sec> secs;
  auto sec_of = [&](QN q) {
    auto it = sidx.find(q.key());
    if (it != sidx.end()) return it->second;
    sidx[q.key()] = int(secs.size());
    secs.push_back(Sec{q, {}, {}, 0, 0});
    return int(secs.size()) - 1;
  };
  std::map<int64_t, std::pair<int, int>> rowpos;  // (sector idx, row idx) per (x, s)
  auto rkey = [](int a, int s) { return int64_t(a) * 64 + s; };
  if (dir > 0) {
    for (size_t a = 0; a < ba.qn.size(); ++a)
      for (int s1 = 0; s1 < d; ++s1) {
        bool any = false;
        for (int s2 = 0; s2 < d && !any; ++s2)
          for (size_t b = 0; b < bb.qn.size() && !any; ++b) any = psi.find(int(a), s1, s2, int(b)) >= 0;
        if (!any) continue;
        const int si = sec_of(ba.qn[a] + ham.q_of_state(s1));
        rowpos[rkey(int(a), s1)] = {si, int(secs[si].rows.size())};
        secs[si].rows.push_back({int(a), s1});
      }
  } else {
    for (int s2 = 0; s2 < d; ++s2)
      for (size_t b = 0; b < bb.qn.size(); ++b) {
        bool any = false;
        for (size_t a = 0; a < ba.qn.size() && !any; ++a)
          for (int s1 = 0; s1 < d && !any; ++s1) any = psi.find(int(a), s1, s2, int(b)) >= 0;
        if (!any) continue;
        const int si = sec_of(bb.qn[b] - ham.q_of_state(s2));
        rowpos[rkey(int(b), s2)] = {si, int(secs[si].rows.size())};
        secs[si].rows.push_back({s2, int(b)});
      }
  }
  // sort sectors by quantum number for a deterministic order
  std::vector<int> sorder(secs.size());
  std::iota(sorder.begin(), sorder.end(), 0);
  std::sort(sorder.begin(), sorder.end(), [&](int i, int j) { return secs[i].q < secs[j].q; });
  int64_t tot = 0;
  for (auto &s : secs) {
    s.roff.resize(s.rows.size());
    int off = 0;
    for (size_t r = 0; r < s.rows.size(); ++r) {
      s.roff[r] = off;
      off += dir > 0 ? ba.dim[s.rows[r].first] : bb.dim[s.rows[r].second];
    }
    s.M = off;
    s.base = tot;
    tot += int64_t(off) * off;
  }
  DevVecs work(dev);
  double *rho = work.get(std::max<int64_t>(1, tot));
  dev_zero(dev, rho, sizeof(double) * std::max<int64_t>(1, tot));
  // rho blocks as grouped GEMM (psi in slot 0, rho in slot 1)
  GemmPlan gp;
  for (auto &s : secs) {
    for (size_t i = 0; i < s.rows.size(); ++i)
      for (size_t j = 0; j < s.rows.size(); ++j) {
        GOut o{};
        o.c_slot = 1;
        o.accumulate = 0;
        o.seg_begin = int32_t(gp.segs.size());
        if (dir > 0) {
          const int a = s.rows[i].first, s1 = s.rows[i].second, a2 = s.rows[j].first, s1b = s.rows[j].second;
          o.c_off = s.base + int64_t(s.roff[i]) * s.M + s.roff[j];
          o.m = ba.dim[a];
          o.n = ba.dim[a2];
          o.ldc = s.M;
          for (int s2 = 0; s2 < d; ++s2)
            for (size_t b = 0; b < bb.qn.size(); ++b) {
              const int p1 = psi.find(a, s1, s2, int(b)), p2 = psi.find(a2, s1b, s2, int(b));
              if (p1 < 0 || p2 < 0) continue;
              GSeg g{};
              g.alpha = rho_scale;
              g.a_slot = 0;
              g.a_off = psi.blk[p1].off;
              g.lda = psi.blk[p1].n;
              g.b_slot = 0;
              g.b_off = psi.blk[p2].off;
              g.ldb = psi.blk[p2].n;
              g.flags = SEG_TB;
              g.k = psi.blk[p1].n;
              gp.segs.push_back(g);
            }
        } else {
          const int s2 = s.rows[i].first, b = s.rows[i].second, s2b = s.rows[j].first, b2 = s.rows[j].second;
          o.c_off = s.base + int64_t(s.roff[i]) * s.M + s.roff[j];
          o.m = bb.dim[b];
          o.n = bb.dim[b2];
          o.ldc = s.M;
          for (size_t a = 0; a < ba.qn.size(); ++a)
            for (int s1 = 0; s1 < d; ++s1) {
              const int p1 = psi.find(int(a), s1, s2, b), p2 = psi.find(int(a), s1, s2b, b2);
              if (p1 < 0 || p2 < 0) continue;
              GSeg g{};
              g.alpha = rho_scale;
              g.a_slot = 0;
              g.a_off = psi.blk[p1].off;
              g.lda = psi.blk[p1].n;
              g.b_slot = 0;
              g.b_off = psi.blk[p2].off;
              g.ldb = psi.blk[p2].n;
              g.flags = SEG_TA;
              g.k = psi.blk[p1].m;
              gp.segs.push_back(g);
            }
        }
        o.seg_count = int32_t(gp.segs.size()) - o.seg_begin;
        if (o.seg_count > 0) gp.outs.push_back(o);
      }
  }
  {
    DevPlan *dp = dev_plan_upload(dev, gp);
    Bases b{};
    for (int i = 0; i < kSlots; ++i) b.p[i] = rho;
    b.p[0] = const_cast<double *>(x);
    b.p[1] = rho;
    dev_gemm_run(dev, dp, b);
    dev_plan_free(dev, dp);
  }
  // eigen-decomposition per sector
  std::vector<std::vector<double>> evals(secs.size());
  int64_t woff = 0;
  std::vector<int64_t> wbase(secs.size());
  for (size_t i = 0; i < secs.size(); ++i) {
    wbase[i] = woff;
    woff += secs[i].M;
  }
  double *wv = work.get(std::max<int64_t>(1, woff));
  for (size_t i = 0; i < secs.size(); ++i) dev_syevd(dev, rho + secs[i].base, secs[i].M, wv + wbase[i]);
  std::vector<double> wall(std::max<int64_t>(1, woff));
  dev_d2h(dev, wall.data(), wv, sizeof(double) * woff);
  work.release(wv);
  // global selection: (-lambda, sector qn, index)
  struct Cand {
    double lam;
    int sec;
    int k;
  };
  std::vector<Cand> cand;
  for (size_t i = 0; i < secs.size(); ++i)
    for (int k = 0; k < secs[i].M; ++k) cand.push_back(Cand{wall[wbase[i] + k], int(i), k});
  std::sort(cand.begin(), cand.end(), [&](const Cand &a, const Cand &b) {
    if (a.lam != b.lam) return a.lam > b.lam;
    if (secs[a.sec].q != secs[b.sec].q) return secs[a.sec].q < secs[b.sec].q;
    return a.k > b.k;
  });
  const int keep = std::min<int>(D, int(cand.size()));
  // weights of the normalised state: rho was formed from x / |x|; dividing
  // by the computed trace as well keeps the weights summing to 1 to rounding
  double tr = 0.0;
  for (const Cand &c : cand) tr += std::max(0.0, c.lam);
  MDMRG_REQUIRE(std::isfinite(tr), -3, "decimate: non-finite density matrix");
  MDMRG_REQUIRE(tr > 0.0, -1, "decimate: zero vector");
  double kept = 0.0, sv = 0.0, sh = 0.0;
  for (size_t i = 0; i < cand.size(); ++i) {
    const double p = std::max(0.0, cand[i].lam) / tr;
    if (int(i) < keep) kept += p;
    if (p > 1e-14) {  // numerical rank: rounding-level eigenvalues excluded
      sv -= p * std::log(p);
      sh += std::sqrt(p);
    }
  }
  if (trunc) *trunc = std::max(0.0, 1.0 - kept);
  if (svn) *svn = sv;
  if (shalf) *shalf = 2.0 * std::log(std::max(sh, 1e-300));
  // kept columns per sector (descending eigenvalue = descending index)
  std::vector<std::vector<int32_t>> kcols(secs.size());
  for (int i = 0; i < keep; ++i) kcols[cand[i].sec].push_back(cand[i].k);
  for (auto &v : kcols) std::sort(v.begin(), v.end(), std::greater<int32_t>());
  // new bond
  Bond nb;
  for (int si : sorder)
    if (!kcols[si].empty()) {
      nb.qn.push_back(secs[si].q);
      nb.dim.push_back(int(kcols[si].size()));
    }
  nb.rebuild_index();
  // new site tensor
  SiteTensor T;
  std::vector<GatherBlk> gb;
  std::vector<int32_t> cols;
  for (int si : sorder) {
    if (kcols[si].empty()) continue;
    const int ni = nb.find(secs[si].q);
    const int cb = int(cols.size());
    cols.insert(cols.end(), kcols[si].begin(), kcols[si].end());
    const Sec &s = secs[si];
    for (size_t r = 0; r < s.rows.size(); ++r) {
      GatherBlk g{};
      g.e_off = s.base;
      g.ldE = s.M;
      g.row0 = s.roff[r];
      g.ncol = int32_t(kcols[si].size());
      g.col_begin = cb;
      if (dir > 0) {
        const int a = s.rows[r].first, s1 = s.rows[r].second;
        g.rows = ba.dim[a];
        T.add(a, s1, ni, int64_t(ba.dim[a]) * nb.dim[ni]);
        g.out_off = T.off.back();
      } else {
        const int s2 = s.rows[r].first, b = s.rows[r].second;
        g.rows = bb.dim[b];
        T.add(ni, s2, b, int64_t(nb.dim[ni]) * bb.dim[b]);
        g.out_off = T.off.back();
      }
      gb.push_back(g);
    }
  }
  T.data = (double *)dev_alloc(dev, sizeof(double) * std::max<int64_t>(1, T.size));
  dev_gather(dev, gb, cols, rho, T.data, dir < 0);
  work.release(rho);
  // install
  const int site = dir > 0 ? l : l + 1;
  if (A[site].data) dev_free(dev, A[site].data);
  A[site] = std::move(T);
  bonds[l + 1] = nb;
  last_decimated = dir;
  // environments that depended on the replaced site / bond are stale
  for (int i = l + 1; i <= ham.n; ++i)
    if (dir > 0 && Lenv[i]) {
      Lenv[i]->release(dev);
      Lenv[i].reset();
    }
  for (int i = 0; i <= l + 1; ++i)
    if (dir < 0 && Renv[i]) {
      Renv[i]->release(dev);
      Renv[i].reset();
    }
  dev_sync(dev);
  stats.t_diag_d += wall_seconds() - t0;
}

// ------------------------------------------------------------- StVec
// dir +1: x_old at bond (l, l+1) with A[l] now a left isometry onto bond
//         l+1; new vector at bond (l+1, l+2) uses A[l+2] (right isometry).
// dir -1: A[l+1] now a right isometry; new vector at bond (l-1, l) uses
//         A[l-1] (left isometry).
void Context::stvec(const double *x_old, int l, int dir, const PsiLayout &ol, double *x_new,
                    const PsiLayout &nl) {
  double t0 = wall_seconds();
  const int d = ham.d;
  // intermediate blocks: dir +1: T[n, s2, b] (bond l+1 sector n, bond l+2 sector b)
  //                      dir -1: T[a, s1, n] (bond l sector a, bond l+1 sector n)
  std::map<std::tuple<int, int, int>, std::pair<int64_t, std::pair<int, int>>> tb;
  int64_t toff = 0;
  GemmPlan p1, p2;
  const Bond &b0 = bonds[l], &b1 = bonds[l + 1], &b2 = bonds[l + 2];
  if (dir > 0) {
    const SiteTensor &Al = A[l];
    for (size_t nsec = 0; nsec < b1.qn.size(); ++nsec)
      for (int s2 = 0; s2 < d; ++s2)
        for (size_t b = 0; b < b2.qn.size(); ++b) {
          GOut o{};
          o.seg_begin = int32_t(p1.segs.size());
          for (size_t a = 0; a < b0.qn.size(); ++a)
            for (int s1 = 0; s1 < d; ++s1) {
              const int ia = Al.find(int(a), s1, int(nsec));
              const int ip = ol.find(int(a), s1, s2, int(b));
              if (ia < 0 || ip < 0) continue;
              GSeg g{};
              g.alpha = 1.0;
              g.a_slot = 6;
              g.a_off = Al.off[ia];
              g.lda = b1.dim[nsec];
              g.flags = SEG_TA;
              g.b_slot = 0;
              g.b_off = ol.blk[ip].off;
              g.ldb = ol.blk[ip].n;
              g.k = b0.dim[a];
              p1.segs.push_back(g);
              p1.flop += 2.0 * b1.dim[nsec] * b2.dim[b] * b0.dim[a];
            }
          o.seg_count = int32_t(p1.segs.size()) - o.seg_begin;
          if (!o.seg_count) continue;
          o.c_slot = 2;
          o.c_off = toff;
          o.m = b1.dim[nsec];
          o.n = b2.dim[b];
          o.ldc = o.n;
          tb[{int(nsec), s2, int(b)}] = {toff, {o.m, o.n}};
          toff += int64_t(o.m) * o.n;
          p1.outs.push_back(o);
        }
    const SiteTensor &B2 = A[l + 2];
    for (const PsiBlk &pb : nl.blk) {  // (n, s2, s3, c)
      GOut o{};
      o.seg_begin = int32_t(p2.segs.size());
      for (size_t b = 0; b < b2.qn.size(); ++b) {
        auto it = tb.find({pb.a, pb.s1, int(b)});
        const int ib = B2.find(int(b), pb.s2, pb.b);
        if (it == tb.end() || ib < 0) continue;
        GSeg g{};
        g.alpha = 1.0;
        g.a_slot = 2;
        g.a_off = it->second.first;
        g.lda = b2.dim[b];
        g.b_slot = 7;
        g.b_off = B2.off[ib];
        g.ldb = pb.n;
        g.k = b2.dim[b];
        p2.segs.push_back(g);
        p2.flop += 2.0 * pb.m * pb.n * b2.dim[b];
      }
      o.seg_count = int32_t(p2.segs.size()) - o.seg_begin;
      o.c_slot = 1;
      o.c_off = pb.off;
      o.m = pb.m;
      o.n = pb.n;
      o.ldc = pb.n;
      o.accumulate = 0;
      p2.outs.push_back(o);
    }
  } else {
    const SiteTensor &Bn = A[l + 1];
    for (size_t a = 0; a < b0.qn.size(); ++a)
      for (int s1 = 0; s1 < d; ++s1)
        for (size_t nsec = 0; nsec < b1.qn.size(); ++nsec) {
          GOut o{};
          o.seg_begin = int32_t(p1.segs.size());
          for (int s2 = 0; s2 < d; ++s2)
            for (size_t b = 0; b < b2.qn.size(); ++b) {
              const int ib = Bn.find(int(nsec), s2, int(b));
              const int ip = ol.find(int(a), s1, s2, int(b));
              if (ib < 0 || ip < 0) continue;
              GSeg g{};
              g.alpha = 1.0;
              g.a_slot = 0;
              g.a_off = ol.blk[ip].off;
              g.lda = ol.blk[ip].n;
              g.b_slot = 6;
              g.b_off = Bn.off[ib];
              g.ldb = b2.dim[b];
              g.flags = SEG_TB;
              g.k = b2.dim[b];
              p1.segs.push_back(g);
              p1.flop += 2.0 * b0.dim[a] * b1.dim[nsec] * b2.dim[b];
            }
          o.seg_count = int32_t(p1.segs.size()) - o.seg_begin;
          if (!o.seg_count) continue;
          o.c_slot = 2;
          o.c_off = toff;
          o.m = b0.dim[a];
          o.n = b1.dim[nsec];
          o.ldc = o.n;
          tb[{int(a), s1, int(nsec)}] = {toff, {o.m, o.n}};
          toff += int64_t(o.m) * o.n;
          p1.outs.push_back(o);
        }
    const SiteTensor &Am = A[l - 1];
    const Bond &bm = bonds[l - 1];
    for (const PsiBlk &pb : nl.blk) {  // (a0, s0, s1, n)
      GOut o{};
      o.seg_begin = int32_t(p2.segs.size());
      for (size_t a = 0; a < b0.qn.size(); ++a) {
        auto it = tb.find({int(a), pb.s2, pb.b});
        const int ia = Am.find(pb.a, pb.s1, int(a));
        if (it == tb.end() || ia < 0) continue;
        GSeg g{};
        g.alpha = 1.0;
        g.a_slot = 7;
        g.a_off = Am.off[ia];
        g.lda = b0.dim[a];
        g.b_slot = 2;
        g.b_off = it->second.first;
        g.ldb = pb.n;
        g.k = b0.dim[a];
        p2.segs.push_back(g);
        p2.flop += 2.0 * pb.m * pb.n * b0.dim[a];
      }
      (void)bm;
      o.seg_count = int32_t(p2.segs.size()) - o.seg_begin;
      o.c_slot = 1;
      o.c_off = pb.off;
      o.m = pb.m;
      o.n = pb.n;
      o.ldc = pb.n;
      o.accumulate = 0;
      p2.outs.push_back(o);
    }
  }
  ensure_scratch(toff);
  dev_zero(dev, x_new, sizeof(double) * nl.n_elem);
  Bases b{};
  for (int i = 0; i < kSlots; ++i) b.p[i] = x_new;
  b.p[0] = const_cast<double *>(x_old);
  b.p[1] = x_new;
  b.p[2] = T_scratch;
  b.p[6] = dir > 0 ? A[l].data : A[l + 1].data;
  b.p[7] = dir > 0 ? A[l + 2].data : A[l - 1].data;
  DevPlan *d1 = dev_plan_upload(dev, p1);
  DevPlan *d2 = dev_plan_upload(dev, p2);
  dev_gemm_run(dev, d1, b);
  dev_gemm_run(dev, d2, b);
  dev_plan_free(dev, d1);
  dev_plan_free(dev, d2);
  dev_sync(dev);
  stats.t_stvec += wall_seconds() - t0;
}

void Context::renormalize(int dir, int prec) {
  MDMRG_REQUIRE(prec >= 0 && prec < kPrecs, -6, "renormalize: unknown precision form");
  MDMRG_REQUIRE(cur >= 0 && last_decimated == dir && (dir == 1 || dir == -1), -4,
                "renormalize: call decimate at the current bond with the same direction first");
  const int l = cur, n = ham.n;
  const int nl = l + dir;
  MDMRG_REQUIRE(nl >= 0 && nl + 1 < n, -1, "renormalize: no bond beyond the chain end");
  double t0 = wall_seconds();
  // the products of this bond are done: its plans, combinations, FP32
  // shadows and graphs are released before the new block is allocated
  // (the wave-function layout is kept for the start vector); until the new
  // bond is prepared there is no current bond, so a failure below leaves a
  // state in which products are refused (ESTATE) until prepare_bond
  const PsiLayout old_psi = psi;
  release_bond();
  ren_prec = prec;
  try {
    if (dir > 0) {
      if (!Lenv[l + 1]) Lenv[l + 1] = renorm_left(*Lenv[l], l);
    } else {
      if (!Renv[l + 1]) Renv[l + 1] = renorm_right(*Renv[l + 2], l + 1);
    }
  } catch (...) {
    ren_prec = 0;
    throw;
  }
  ren_prec = 0;
  // no wait here: the host part of the next bond's Tables step overlaps
  // these launches (its first plan upload waits for the stream), so Ren
  // counts the host side of the renormalisation and Tables the rest
  stats.t_ren += wall_seconds() - t0;
  prev_psi = old_psi;
  prev_l = l;
  prev_dir = dir;
  prepare(nl);
  last_decimated = 0;
}

// ------------------------------------------------------------- sweeps
int Context::sweep(int n_sweeps, const int *Ds, int n_sched, double tol, double *energies) {
  MDMRG_REQUIRE(have_ham && have_mps, -4, "sweep: Hamiltonian and MPS required");
  MDMRG_REQUIRE(n_sweeps >= 1 && n_sched >= 1, -1, "sweep: bad schedule");
  const int n = ham.n;
  MDMRG_REQUIRE(n >= 3, -1, "sweep: need at least 3 sites");
  // start at bond (0, 1)
  prepare(0);
  DevVecs vecs(dev);
  double *x = vecs.get(std::max<int64_t>(1, psi.n_elem));
  dev_randn(dev, x, psi.n_elem, 1);
  double e = 0.0;
  int not_converged = 0;
  for (int sw = 0; sw < n_sweeps; ++sw) {
    const int D = Ds[std::min(sw, n_sched - 1)];
    for (int dir : {1, -1}) {
      const int lo = 0, hi = n - 2;
      int l = dir > 0 ? lo : hi;
      while (true) {
        double res;
        int nmv;
        if (davidson(x, tol, 200, 24, &e, &res, &nmv) != 0) ++not_converged;
        const bool last = dir > 0 ? (l == hi - 1) : (l == lo + 1);
        decimate(x, D, dir, nullptr, nullptr, nullptr);
        renormalize(dir);
        double *xn = vecs.get(std::max<int64_t>(1, psi.n_elem));
        stvec(x, prev_l, dir, prev_psi, xn, psi);
        vecs.release(x);
        x = xn;
        l = cur;
        if (last) {
          // the turning bond is optimised at the start of the next half-sweep
          break;
        }
      }
    }
    if (energies) energies[sw] = e;
  }
  vecs.release(x);
  dev_sync(dev);
  // every bond was still decimated and the sweep completed; a Davidson solve
  // that missed tol makes the sweep report ENOCONV
  if (not_converged) err = "sweep: " + std::to_string(not_converged) + " Davidson solve(s) did not reach tol";
  return not_converged ? -5 : 0;
}

}  // namespace mdmrg
