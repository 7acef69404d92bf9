// extern "C" boundary of libmdmrg: argument checks, exception -> status.
#include <algorithm>
#include <cmath>
#include <memory>

#include "../../include/mdmrg.h"
#include "engine.h"

using namespace mdmrg;

struct mdmrg_ctx_s {
  Context c;
};

template <class F>
static int guarded(mdmrg_ctx ctx, F &&f) {
  try {
    if (ctx) ctx->c.err.clear();
    return f();
  } catch (const Error &e) {
    if (ctx) ctx->c.err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    if (ctx) ctx->c.err = "host allocation failed";
    return MDMRG_ENOMEM;
  } catch (const std::exception &e) {
    if (ctx) ctx->c.err = e.what();
    return MDMRG_EDEVICE;
  }
}

// Message of the last failed call that has no context (creation, the host
// analysis functions); per thread.
namespace mdmrg {
thread_local std::string g_err;
}

extern "C" {

const char *mdmrg_version(void) { return "mdmrg 0.1 (gfx950)"; }

int mdmrg_create(mdmrg_ctx *out, int device, void *hip_stream) {
  if (!out) return MDMRG_EINVAL;
  *out = nullptr;
  try {
    std::unique_ptr<mdmrg_ctx_s> c(new mdmrg_ctx_s());
    c->c.dev = dev_create(device, hip_stream);
    dev_timing_enable(c->c.dev, true);
    *out = c.release();
    return MDMRG_OK;
  } catch (const Error &e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return MDMRG_ENOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return MDMRG_EDEVICE;
  }
}

void mdmrg_destroy(mdmrg_ctx ctx) { delete ctx; }

const char *mdmrg_last_error(mdmrg_ctx ctx) { return ctx ? ctx->c.err.c_str() : g_err.c_str(); }

int mdmrg_lattice_nso(int model, int Lx, int Ly) {
  if (Lx < 1 || Ly < 1 || (model != 0 && model != 1)) return MDMRG_EINVAL;
  return lattice_nso(model, Lx, Ly);
}

int mdmrg_build_lattice(int model, int basis, int Lx, int Ly, double t, double u, double *T, double *V) {
  if (!T || !V) return MDMRG_EINVAL;
  return guarded(nullptr, [&] {
    build_lattice(model, basis, Lx, Ly, t, u, T, V);
    return MDMRG_OK;
  });
}

int mdmrg_rotate_modes(int n_modes, int spin_half, const double *R, double *T, double *V) {
  if (!R || !T || !V || n_modes < 1) return MDMRG_EINVAL;
  return guarded(nullptr, [&] {
    rotate_modes(n_modes, spin_half, R, T, V);
    return MDMRG_OK;
  });
}

static int set_ham(mdmrg_ctx ctx, int n_sites, int spin_half, const double *T, const double *V,
                   const int32_t *ijkl, const double *val, int64_t nnz, int ta, int tb) {
  if (!ctx) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    MDMRG_REQUIRE(n_sites >= 2 && T, MDMRG_EINVAL, "set_hamiltonian: bad arguments");
    Context &c = ctx->c;
    c.reset_envs();
    c.have_mps = false;
    c.ham.build(n_sites, spin_half, T, V, ijkl, val, nnz, QN(ta, spin_half ? tb : 0));
    c.have_ham = true;
    return MDMRG_OK;
  });
}

int mdmrg_set_hamiltonian(mdmrg_ctx ctx, int n_sites, int spin_half, const double *T, const double *V,
                          int target_a, int target_b) {
  if (!V) return MDMRG_EINVAL;
  return set_ham(ctx, n_sites, spin_half, T, V, nullptr, nullptr, 0, target_a, target_b);
}

int mdmrg_set_hamiltonian_coo(mdmrg_ctx ctx, int n_sites, int spin_half, const double *T, int64_t nnz,
                              const int32_t *ijkl, const double *val, int target_a, int target_b) {
  if (nnz < 0 || (nnz > 0 && (!ijkl || !val))) return MDMRG_EINVAL;
  return set_ham(ctx, n_sites, spin_half, T, nullptr, ijkl, val, nnz, target_a, target_b);
}

int mdmrg_n_terms(mdmrg_ctx ctx, int64_t *n1, int64_t *n2) {
  if (!ctx) return MDMRG_EINVAL;
  if (!ctx->c.have_ham) return MDMRG_ESTATE;
  if (n1) *n1 = ctx->c.ham.n1;
  if (n2) *n2 = ctx->c.ham.n2;
  return MDMRG_OK;
}

int mdmrg_set_mps(mdmrg_ctx ctx, const int32_t *n_sect, const int32_t *sect_qn, const int32_t *sect_dim,
                  const double *data, int64_t n_data) {
  if (!ctx || !n_sect || !sect_qn || !sect_dim || (!data && n_data)) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    Context &c = ctx->c;
    MDMRG_REQUIRE(c.have_ham, MDMRG_ESTATE, "set_mps: set the Hamiltonian first");
    const int n = c.ham.n, d = c.ham.d;
    c.reset_envs();
    for (auto &t : c.A)
      if (t.data) dev_free(c.dev, t.data);
    c.A.clear();
    c.bonds.assign(n + 1, Bond());
    int64_t s = 0;
    for (int i = 0; i <= n; ++i) {
      MDMRG_REQUIRE(n_sect[i] >= 1, MDMRG_EINVAL, "set_mps: every bond needs a sector");
      for (int k = 0; k < n_sect[i]; ++k, ++s) {
        const QN q(sect_qn[2 * s], sect_qn[2 * s + 1]);
        MDMRG_REQUIRE(sect_dim[s] >= 1, MDMRG_EINVAL, "set_mps: sector dimensions must be positive");
        if (!c.bonds[i].qn.empty())
          MDMRG_REQUIRE(c.bonds[i].qn.back() < q, MDMRG_EINVAL, "set_mps: sectors must be strictly ascending");
        c.bonds[i].qn.push_back(q);
        c.bonds[i].dim.push_back(sect_dim[s]);
      }
      c.bonds[i].rebuild_index();
    }
    MDMRG_REQUIRE(c.bonds[0].qn.size() == 1 && c.bonds[0].qn[0] == QN() && c.bonds[0].dim[0] == 1,
                  MDMRG_EINVAL, "set_mps: bond 0 must be the vacuum");
    MDMRG_REQUIRE(c.bonds[n].qn.size() == 1 && c.bonds[n].qn[0] == c.ham.target && c.bonds[n].dim[0] == 1,
                  MDMRG_EINVAL, "set_mps: last bond must be the target sector");
    int64_t pos = 0;
    c.A.resize(n);
    for (int i = 0; i < n; ++i) {
      SiteTensor &T = c.A[i];
      const Bond &L = c.bonds[i], &R = c.bonds[i + 1];
      for (size_t l = 0; l < L.qn.size(); ++l)
        for (int st = 0; st < d; ++st) {
          const int r = R.find(L.qn[l] + c.ham.q_of_state(st));
          if (r < 0) continue;
          T.add(int(l), st, r, int64_t(L.dim[l]) * R.dim[r]);
        }
      MDMRG_REQUIRE(pos + T.size <= n_data, MDMRG_EINVAL, "set_mps: data shorter than the sector layout");
      T.data = (double *)dev_alloc(c.dev, sizeof(double) * std::max<int64_t>(1, T.size));
      dev_h2d(c.dev, T.data, data + pos, sizeof(double) * T.size);
      pos += T.size;
    }
    MDMRG_REQUIRE(pos == n_data, MDMRG_EINVAL, "set_mps: data longer than the sector layout");
    c.have_mps = true;
    return MDMRG_OK;
  });
}

int mdmrg_get_mps(mdmrg_ctx ctx, double *data, int64_t n_data, int64_t *n_needed) {
  if (!ctx) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    Context &c = ctx->c;
    MDMRG_REQUIRE(c.have_mps, MDMRG_ESTATE, "get_mps: no MPS");
    const int n = c.ham.n, d = c.ham.d;
    // the exchange layout of mdmrg_set_mps: site by site, blocks (l, s, r)
    // in lexicographic order, each row-major; absent blocks are zero
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
      const Bond &L = c.bonds[i], &R = c.bonds[i + 1];
      for (size_t l = 0; l < L.qn.size(); ++l)
        for (int st = 0; st < d; ++st) {
          const int r = R.find(L.qn[l] + c.ham.q_of_state(st));
          if (r >= 0) total += int64_t(L.dim[l]) * R.dim[r];
        }
    }
    if (n_needed) *n_needed = total;
    if (!data) return MDMRG_OK;
    MDMRG_REQUIRE(n_data >= total, MDMRG_EINVAL, "get_mps: data shorter than the sector layout");
    int64_t pos = 0;
    for (int i = 0; i < n; ++i) {
      const Bond &L = c.bonds[i], &R = c.bonds[i + 1];
      const SiteTensor &T = c.A[i];
      for (size_t l = 0; l < L.qn.size(); ++l)
        for (int st = 0; st < d; ++st) {
          const int r = R.find(L.qn[l] + c.ham.q_of_state(st));
          if (r < 0) continue;
          const int64_t sz = int64_t(L.dim[l]) * R.dim[r];
          const int b = T.find(int(l), st, r);
          if (b >= 0 && T.data)
            dev_d2h(c.dev, data + pos, T.data + T.off[b], sizeof(double) * sz);
          else
            std::fill(data + pos, data + pos + sz, 0.0);
          pos += sz;
        }
    }
    return MDMRG_OK;
  });
}

int mdmrg_get_bond(mdmrg_ctx ctx, int bond, int32_t *n_sect, int32_t *qn, int32_t *dim) {
  if (!ctx || !n_sect) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    Context &c = ctx->c;
    MDMRG_REQUIRE(c.have_mps, MDMRG_ESTATE, "get_bond: no MPS");
    MDMRG_REQUIRE(bond >= 0 && bond <= c.ham.n, MDMRG_EINVAL, "get_bond: bond out of range");
    const Bond &b = c.bonds[bond];
    *n_sect = int32_t(b.qn.size());
    for (size_t i = 0; i < b.qn.size(); ++i) {
      if (qn) {
        qn[2 * i] = b.qn[i].a;
        qn[2 * i + 1] = b.qn[i].b;
      }
      if (dim) dim[i] = b.dim[i];
    }
    return MDMRG_OK;
  });
}

int mdmrg_set_option(mdmrg_ctx ctx, int option, int64_t value) {
  if (!ctx) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    Context &c = ctx->c;
    switch (option) {
      case MDMRG_OPT_KEEP_ENVS:
        MDMRG_REQUIRE(value >= 0 && value <= 3, MDMRG_EINVAL, "set_option: keep-envs mode must be 0..3");
        c.keep_envs = int(value);
        break;
      case MDMRG_OPT_SCRATCH_LIMIT:
        MDMRG_REQUIRE(value >= (int64_t(1) << 20), MDMRG_EINVAL, "set_option: scratch limit below 2^20 doubles");
        c.scratch_limit = value;
        break;
      case MDMRG_OPT_GRAPH:
        c.set_graph(value != 0);
        break;
      case MDMRG_OPT_COMPRESS:
        c.compress = value != 0;
        break;
      case MDMRG_OPT_MEMORY_BUDGET:
        MDMRG_REQUIRE(value >= 0, MDMRG_EINVAL, "set_option: negative memory budget");
        dev_set_budget(c.dev, size_t(value));
        break;
      case MDMRG_OPT_DAVIDSON_KEEP:
        MDMRG_REQUIRE(value >= 2 && value <= 58, MDMRG_EINVAL, "set_option: Davidson restart size must be 2..58");
        c.davidson_keep = int(value);
        break;
      case MDMRG_OPT_DAVIDSON_OLSEN:
        c.davidson_olsen = value != 0;
        break;
      case MDMRG_OPT_MIXED_LADDER:
        c.mixed_ladder = value != 0;
        break;
      case MDMRG_OPT_MIXED_CORRECT:
        c.mixed_correct = value != 0;
        break;
      case MDMRG_OPT_MIXED_HANDOVER:
        MDMRG_REQUIRE(value >= 1 && value <= 16, MDMRG_EINVAL, "set_option: hand-over size must be 1..16");
        c.mixed_handover = int(value);
        break;
      case MDMRG_OPT_GEMM_VARIANT:
        MDMRG_REQUIRE(value >= -1 && value < kGemmVariants, MDMRG_EINVAL, "set_option: no such tile variant");
        dev_force_variant(c.dev, int(value));
        break;
      default:
        throw Error(MDMRG_EINVAL, "set_option: unknown option");
    }
    return MDMRG_OK;
  });
}

int mdmrg_prepare_bond(mdmrg_ctx ctx, int l) {
  if (!ctx) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    ctx->c.prepare(l);
    return MDMRG_OK;
  });
}

int mdmrg_psi_layout(mdmrg_ctx ctx, int64_t *n_elem, int32_t *n_blk, int32_t *desc) {
  if (!ctx) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    Context &c = ctx->c;
    MDMRG_REQUIRE(c.cur >= 0, MDMRG_ESTATE, "psi_layout: no current bond");
    if (n_elem) *n_elem = c.psi.n_elem;
    if (n_blk) *n_blk = int32_t(c.psi.blk.size());
    if (desc)
      for (size_t i = 0; i < c.psi.blk.size(); ++i) {
        const PsiBlk &b = c.psi.blk[i];
        int32_t *o = desc + 8 * i;
        o[0] = b.a;
        o[1] = b.s1;
        o[2] = b.s2;
        o[3] = b.b;
        o[4] = b.m;
        o[5] = b.n;
        o[6] = int32_t(b.off & 0xffffffff);
        o[7] = int32_t(b.off >> 32);
      }
    return MDMRG_OK;
  });
}

int mdmrg_heff_apply(mdmrg_ctx ctx, int prec, const double *x, double *y) {
  if (!ctx || !x || !y || x == y) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    MDMRG_REQUIRE(prec == MDMRG_FP64 || prec == MDMRG_FP32 || prec == MDMRG_BF16X3 || prec == MDMRG_BF16X6, MDMRG_EUNSUP,
                  "heff_apply: unknown precision form");
    ctx->c.heff_apply(x, y, prec);
    dev_sync(ctx->c.dev);
    return MDMRG_OK;
  });
}

int mdmrg_heff_diag(mdmrg_ctx ctx, double *d) {
  if (!ctx || !d) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    ctx->c.heff_diag(d);
    dev_sync(ctx->c.dev);
    return MDMRG_OK;
  });
}

int mdmrg_heff_cost(mdmrg_ctx ctx, double *flop, double *bytes, int64_t *n_terms, int64_t *n_gemm) {
  if (!ctx) return MDMRG_EINVAL;
  if (ctx->c.cur < 0) return MDMRG_ESTATE;
  if (flop) *flop = ctx->c.heff.flop;
  if (bytes) *bytes = ctx->c.heff.bytes;
  if (n_terms) *n_terms = ctx->c.heff_terms;
  if (n_gemm) *n_gemm = ctx->c.heff.n_gemm;
  return MDMRG_OK;
}

int mdmrg_heff_histogram(mdmrg_ctx ctx, double *flop_by_bin) {
  if (!ctx || !flop_by_bin) return MDMRG_EINVAL;
  if (ctx->c.cur < 0) return MDMRG_ESTATE;
  for (int b = 0; b < TwoPhasePlan::kHistBins; ++b) flop_by_bin[b] = ctx->c.heff.hist_flop[b];
  return MDMRG_OK;
}

int mdmrg_davidson(mdmrg_ctx ctx, double *x, double tol, int max_iter, int m_max, double *energy, double *resid,
                   int *n_matvec) {
  if (!ctx || !x || !(tol > 0) || max_iter < 1) return MDMRG_EINVAL;
  return guarded(ctx, [&] { return ctx->c.davidson(x, tol, max_iter, m_max, energy, resid, n_matvec); });
}

int mdmrg_davidson_mixed(mdmrg_ctx ctx, double *x, double tol, int prec_split, double tol_split, int max_iter,
                         int m_max, double *energy, double *resid, int *n_mv64, int *n_mv_split) {
  if (!ctx || !x || !(tol > 0) || !(tol_split > 0) || max_iter < 1) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    return ctx->c.davidson_mixed(x, tol, prec_split, tol_split, max_iter, m_max, energy, resid, n_mv64,
                                 n_mv_split);
  });
}

int mdmrg_decimate(mdmrg_ctx ctx, const double *x, int D, int direction, double *trunc_err, double *s_vn,
                   double *s_half) {
  if (!ctx || !x) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    ctx->c.decimate(x, D, direction, trunc_err, s_vn, s_half);
    return MDMRG_OK;
  });
}

int mdmrg_renormalize(mdmrg_ctx ctx, int direction, int prec) {
  if (!ctx) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    MDMRG_REQUIRE(prec == MDMRG_FP64 || prec == MDMRG_FP32 || prec == MDMRG_BF16X3 || prec == MDMRG_BF16X6, MDMRG_EUNSUP,
                  "renormalize: unknown precision form");
    ctx->c.renormalize(direction, prec);
    return MDMRG_OK;
  });
}

int mdmrg_stvec(mdmrg_ctx ctx, const double *x_old, double *x_new) {
  if (!ctx || !x_old || !x_new || x_old == x_new) return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    Context &c = ctx->c;
    MDMRG_REQUIRE(c.prev_l >= 0 && c.cur == c.prev_l + c.prev_dir, MDMRG_ESTATE,
                  "stvec: call renormalize first");
    c.stvec(x_old, c.prev_l, c.prev_dir, c.prev_psi, x_new, c.psi);
    return MDMRG_OK;
  });
}

int mdmrg_sweep(mdmrg_ctx ctx, int n_sweeps, const int *D_schedule, int n_sched, double tol, double *energies) {
  if (!ctx || !D_schedule) return MDMRG_EINVAL;
  return guarded(ctx, [&] { return ctx->c.sweep(n_sweeps, D_schedule, n_sched, tol, energies); });
}

// Descriptor check and launch shared by the FP64 and FP32-buffer forms of
// the grouped GEMM: offsets and lengths are in elements of the buffers.
static int gemm_grouped_any(mdmrg_ctx ctx, int prec, int n_bases, void *const *bases, const int64_t *base_len,
                            int64_t n_out, const int64_t *out_desc, int64_t n_seg, const int64_t *seg_desc,
                            const double *alpha, bool noalloc = false) {
  if (!ctx || n_bases < 1 || n_bases > kSlots || !bases || !base_len || n_out < 0 || n_seg < 0 ||
      (n_out && !out_desc) || (n_seg && (!seg_desc || !alpha)))
    return MDMRG_EINVAL;
  return guarded(ctx, [&] {
    GemmPlan plan;
    auto in_range = [&](int slot, int64_t off, int64_t last) {
      return slot >= 0 && slot < n_bases && off >= 0 && last >= 0 && off + last < base_len[slot];
    };
    for (int64_t e = 0; e < n_seg; ++e) {
      const int64_t *d = seg_desc + 8 * e;
      GSeg g{};
      g.a_slot = uint8_t(d[0]);
      g.a_off = d[1];
      g.lda = int32_t(d[2]);
      g.b_slot = uint8_t(d[3]);
      g.b_off = d[4];
      g.ldb = int32_t(d[5]);
      g.k = int32_t(d[6]);
      g.flags = uint8_t(d[7] & 7);
      g.alpha = alpha[e];
      MDMRG_REQUIRE(d[6] >= 0 && d[6] < (int64_t(1) << 31) && d[2] >= 0 && d[5] >= 0 && d[0] < kSlots &&
                        d[3] < kSlots && d[0] >= 0 && d[3] >= 0,
                    MDMRG_EINVAL, "gemm_grouped: bad segment descriptor");
      plan.segs.push_back(g);
    }
    for (int64_t o = 0; o < n_out; ++o) {
      const int64_t *d = out_desc + 8 * o;
      GOut g{};
      g.c_slot = uint8_t(d[0]);
      g.c_off = d[1];
      g.m = int32_t(d[2]);
      g.n = int32_t(d[3]);
      g.ldc = int32_t(d[4]);
      g.seg_begin = int32_t(d[5]);
      g.seg_count = int32_t(d[6]);
      g.accumulate = uint8_t(d[7] != 0);
      MDMRG_REQUIRE(d[2] >= 1 && d[3] >= 1 && d[4] >= d[3] && d[2] < (1 << 30) && d[3] < (1 << 30) &&
                        d[4] < (int64_t(1) << 31) &&
                        d[5] >= 0 && d[6] >= 0 && d[5] + d[6] <= n_seg,
                    MDMRG_EINVAL, "gemm_grouped: bad output descriptor");
      MDMRG_REQUIRE(in_range(int(d[0]), d[1], (d[2] - 1) * d[4] + d[3] - 1), MDMRG_EINVAL,
                    "gemm_grouped: output block outside its buffer");
      for (int64_t q = d[5]; q < d[5] + d[6]; ++q) {
        const GSeg &sg = plan.segs[q];
        const int64_t m = d[2], n = d[3], k = sg.k;
        if (k == 0) continue;
        if (!(sg.flags & SEG_AID)) {
          const int64_t last = (sg.flags & SEG_TA) ? (k - 1) * sg.lda + m - 1 : (m - 1) * sg.lda + k - 1;
          MDMRG_REQUIRE(in_range(sg.a_slot, sg.a_off, last) && sg.lda >= ((sg.flags & SEG_TA) ? m : k),
                        MDMRG_EINVAL, "gemm_grouped: A operand outside its buffer");
        }
        const int64_t lastb = (sg.flags & SEG_TB) ? (n - 1) * sg.ldb + k - 1 : (k - 1) * sg.ldb + n - 1;
        MDMRG_REQUIRE(in_range(sg.b_slot, sg.b_off, lastb) && sg.ldb >= ((sg.flags & SEG_TB) ? k : n),
                      MDMRG_EINVAL, "gemm_grouped: B operand outside its buffer");
        if (!(sg.flags & SEG_AID)) plan.flop += 2.0 * m * n * k;
      }
      plan.outs.push_back(g);
    }
    Bases b{};
    for (int i = 0; i < kSlots; ++i) b.p[i] = static_cast<double *>(bases[i < n_bases ? i : 0]);
    if (noalloc) {
      dev_gemm_run_noalloc(ctx->c.dev, plan, b);  // waits for the launch
      return MDMRG_OK;
    }
    DevPlan *dp = dev_plan_upload(ctx->c.dev, plan);
    dev_gemm_run(ctx->c.dev, dp, b, 3, prec);
    dev_plan_free(ctx->c.dev, dp);
    dev_sync(ctx->c.dev);
    return MDMRG_OK;
  });
}

int mdmrg_gemm_grouped(mdmrg_ctx ctx, int n_bases, const double *const *bases, const int64_t *base_len,
                       int64_t n_out, const int64_t *out_desc, int64_t n_seg, const int64_t *seg_desc,
                       const double *alpha) {
  if (!bases) return MDMRG_EINVAL;
  void *p[kSlots] = {};
  for (int i = 0; i < n_bases && i < kSlots; ++i) p[i] = const_cast<double *>(bases[i]);
  return gemm_grouped_any(ctx, MDMRG_FP64, n_bases, p, base_len, n_out, out_desc, n_seg, seg_desc, alpha);
}

static_assert(kNoAllocStagingBytes == MDMRG_NOALLOC_STAGING_BYTES, "staging size of the header and the device layer");

int mdmrg_gemm_grouped_noalloc(mdmrg_ctx ctx, int n_bases, const double *const *bases, const int64_t *base_len,
                               int64_t n_out, const int64_t *out_desc, int64_t n_seg, const int64_t *seg_desc,
                               const double *alpha) {
  if (!bases) return MDMRG_EINVAL;
  void *p[kSlots] = {};
  for (int i = 0; i < n_bases && i < kSlots; ++i) p[i] = const_cast<double *>(bases[i]);
  return gemm_grouped_any(ctx, MDMRG_FP64, n_bases, p, base_len, n_out, out_desc, n_seg, seg_desc, alpha, true);
}

int mdmrg_gemm_grouped_split(mdmrg_ctx ctx, int prec, int n_bases, const float *const *bases,
                             const int64_t *base_len, int64_t n_out, const int64_t *out_desc, int64_t n_seg,
                             const int64_t *seg_desc, const double *alpha) {
  if (!ctx || !bases) return MDMRG_EINVAL;
  if (prec != MDMRG_FP32 && prec != MDMRG_BF16X3 && prec != MDMRG_BF16X6) {
    ctx->c.err = "gemm_grouped_split: prec must be MDMRG_FP32, MDMRG_BF16X3 or MDMRG_BF16X6";
    return MDMRG_EUNSUP;
  }
  void *p[kSlots] = {};
  for (int i = 0; i < n_bases && i < kSlots; ++i) p[i] = const_cast<float *>(bases[i]);
  return gemm_grouped_any(ctx, prec, n_bases, p, base_len, n_out, out_desc, n_seg, seg_desc, alpha);
}

int mdmrg_get_stats(mdmrg_ctx ctx, double *out) {
  if (!ctx || !out) return MDMRG_EINVAL;
  const Stats &s = ctx->c.stats;
  out[0] = s.t_diag_h;
  out[1] = s.t_ren;
  out[2] = s.t_tables;
  out[3] = s.t_diag_d;
  out[4] = s.t_stvec;
  out[5] = s.t_other;
  out[6] = s.heff_flop;
  out[7] = s.n_matvec;
  return guarded(ctx, [&] {
    double ms[kTags], ln[kTags], fl[kTags];
    dev_timing_collect(ctx->c.dev, ms, ln, fl);
    out[8] = ms[1];
    out[9] = ln[1];
    out[10] = fl[1];
    out[11] = ms[2];
    out[12] = ln[2];
    out[13] = fl[2];
    out[14] = s.heff_flop_split;
    out[15] = s.n_matvec_split;
    out[16] = ms[4];
    out[17] = ln[4];
    out[18] = fl[4];
    out[19] = ms[5];
    out[20] = ln[5];
    out[21] = fl[5];
    out[22] = ms[3];
    out[23] = ln[3];
    out[24] = fl[3];
    // FP64 H_eff products (both phases), then every launch of the context
    out[25] = ms[1] + ms[5];
    out[26] = ln[1] + ln[5];
    out[27] = fl[1] + fl[5];
    out[28] = out[29] = 0.0;
    for (int i = 1; i < kTags; ++i) {
      out[28] += ms[i];
      out[29] += ln[i];
    }
    double pm[kPrecs][kGemmVariants], pl[kPrecs][kGemmVariants], pf[kPrecs][kGemmVariants];
    dev_timing_process(ctx->c.dev, pm, pl, pf);
    for (int p = 0; p < kPrecs; ++p)
      for (int v = 0; v < kGemmVariants; ++v) {
        const int at = 30 + 3 * (kGemmVariants * p + v);
        out[at] = pm[p][v];
        out[at + 1] = pl[p][v];
        out[at + 2] = pf[p][v];
      }
    constexpr int g = 30 + 3 * kGemmVariants * kPrecs;
    static_assert(g + 2 * kPrecs == MDMRG_N_STATS, "stats layout");
    for (int p = 0; p < kPrecs; ++p) {
      out[g + 2 * p] = ms[7 + p];
      out[g + 2 * p + 1] = ln[7 + p];
    }
    return MDMRG_OK;
  });
}

}  // extern "C"
