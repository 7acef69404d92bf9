// Host analysis of a matrix product state at the end of a sweep (Sec. II.B):
// the one- and two-mode reduced density operators and their von Neumann
// entropies, the one-particle density matrix, occupations and density
// correlations (with the CDW order parameter of Sec. III.C), the mutual
// information with the total correlation and correlation distance, the
// natural modes, the Fiedler ordering, the DEAS order and the HF reference
// configuration that set up the next mode-transformation macro-iteration;
// and the two-mode micro-iterations that build the mode transformation
// (the S_1/2-minimising rotation of a bond's two modes, and a sweep of them
// through the chain with the composite rotation).
//
// Everything here runs on the host from the MPS exchange arrays (the format
// of mdmrg_set_mps / mdmrg_get_mps); no context and no GPU are involved.
//
// Mode density operators.  The MPS amplitude of the local configurations
// (s_0 .. s_{n-1}) is the coefficient of the Fock state with the creation
// operators in chain order.  For modes i < j the density operator in the
// representation with the modes' spin-orbitals moved to the front (i's first)
// is
//   rho[(c,e),(c',e')] = sum_rest psi(..c..e..) psi(..c'..e'..) (-1)^{P}
// where P = (N(e) + N(e')) * (particles on the sites strictly between i and
// j): the Jordan-Wigner string of the reordering.  It is contracted left to
// right: the left environment E_L[i] (sum over the configurations of sites
// < i), the pair (c, c') at site i, the transfer over sites i+1 .. j-1 (with
// the parity of each site's state when N(c) + N(c') is odd), the pair
// (e, e') at site j and the right environment E_R[j+1].  Every operator
// between two bonds maps a bra sector to one ket sector (its quantum-number
// shift is fixed), so it is stored as one dense block per bra sector.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <exception>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mdmrg.h"

namespace mdmrg {
extern thread_local std::string g_err;  // read by mdmrg_last_error(NULL)
}

namespace {

struct BadInput : std::runtime_error {
  using std::runtime_error::runtime_error;
};

struct Mps {
  int n = 0, ns = 1, d = 2;
  std::vector<std::vector<std::array<int, 2>>> qn;  // per bond
  std::vector<std::vector<int>> dim;                // per bond
  // per site: block of (l, s) -> (r, offset) or r = -1
  std::vector<std::vector<int>> blk_r;
  std::vector<std::vector<int64_t>> blk_off;
  std::vector<int64_t> site_off;  // data of site i: [site_off[i], site_off[i+1])
  const double *data = nullptr;

  std::array<int, 2> q(int s) const {
    return ns == 2 ? std::array<int, 2>{s & 1, (s >> 1) & 1} : std::array<int, 2>{s & 1, 0};
  }
  int find(int bond, std::array<int, 2> Q) const {
    const auto &v = qn[bond];
    auto it = std::lower_bound(v.begin(), v.end(), Q);
    return (it != v.end() && *it == Q) ? int(it - v.begin()) : -1;
  }
};

void parse(Mps &m, int n_sites, int spin_half, const int32_t *n_sect, const int32_t *sect_qn,
           const int32_t *sect_dim, const double *data, int64_t n_data) {
  m.n = n_sites;
  m.ns = spin_half ? 2 : 1;
  m.d = 1 << m.ns;
  m.data = data;
  m.qn.resize(n_sites + 1);
  m.dim.resize(n_sites + 1);
  int64_t k = 0;
  for (int b = 0; b <= n_sites; ++b) {
    if (n_sect[b] < 1) throw BadInput("a bond has no sectors");
    for (int t = 0; t < n_sect[b]; ++t, ++k) {
      std::array<int, 2> Q{sect_qn[2 * k], sect_qn[2 * k + 1]};
      if (sect_dim[k] < 1) throw BadInput("a sector has dimension < 1");
      if (t > 0 && !(m.qn[b].back() < Q)) throw BadInput("sectors not in ascending order");
      m.qn[b].push_back(Q);
      m.dim[b].push_back(sect_dim[k]);
    }
  }
  if (m.qn[0].size() != 1 || m.qn[0][0] != std::array<int, 2>{0, 0} || m.dim[0][0] != 1 ||
      m.qn[n_sites].size() != 1 || m.dim[n_sites][0] != 1)
    throw BadInput("bond 0 must be {(0,0): 1} and bond n a single sector of dimension 1");
  int64_t off = 0;
  m.blk_r.resize(n_sites);
  m.blk_off.resize(n_sites);
  m.site_off.assign(n_sites + 1, 0);
  for (int i = 0; i < n_sites; ++i) {
    m.site_off[i] = off;
    const int nl = int(m.qn[i].size());
    m.blk_r[i].assign(size_t(nl) * m.d, -1);
    m.blk_off[i].assign(size_t(nl) * m.d, -1);
    for (int l = 0; l < nl; ++l)
      for (int s = 0; s < m.d; ++s) {
        const auto qs = m.q(s);
        const int r = m.find(i + 1, {m.qn[i][l][0] + qs[0], m.qn[i][l][1] + qs[1]});
        if (r < 0) continue;
        m.blk_r[i][size_t(l) * m.d + s] = r;
        m.blk_off[i][size_t(l) * m.d + s] = off;
        off += int64_t(m.dim[i][l]) * m.dim[i + 1][r];
      }
  }
  m.site_off[n_sites] = off;
  if (off != n_data) throw BadInput("n_data does not match the sector layout");
}

// An operator between the bra and ket copies of one bond: per bra sector
// the ket sector (-1: none) and a dense m_bra x m_ket block, row-major.
struct Op {
  std::vector<int> ket;
  std::vector<std::vector<double>> mat;
};

Op identity_op(const Mps &m, int bond, double scale = 1.0) {
  Op o;
  const int ns = int(m.qn[bond].size());
  o.ket.resize(ns);
  o.mat.resize(ns);
  for (int t = 0; t < ns; ++t) {
    o.ket[t] = t;
    const int md = m.dim[bond][t];
    o.mat[t].assign(size_t(md) * md, 0.0);
    for (int a = 0; a < md; ++a) o.mat[t][size_t(a) * md + a] = scale;
  }
  return o;
}

// X' = sum A^{sb T} X A^{sk} over site i: (sb, sk) fixed when sb >= 0,
// otherwise summed over s = sb = sk with the sign (-1)^{N(s)} when parity.
Op apply_site(const Mps &m, int i, const Op &X, int sb, int sk, bool parity) {
  const int nr = int(m.qn[i + 1].size());
  Op out;
  out.ket.assign(nr, -1);
  out.mat.resize(nr);
  std::vector<double> tmp;
  const int nl = int(m.qn[i].size());
  for (int l = 0; l < nl; ++l) {
    const int lk = X.ket[l];
    if (lk < 0) continue;
    const int s0 = sb >= 0 ? sb : 0, s1 = sb >= 0 ? sb + 1 : m.d;
    for (int s = s0; s < s1; ++s) {
      const int sK = sb >= 0 ? sk : s;
      const int r = m.blk_r[i][size_t(l) * m.d + s];
      const int rk = m.blk_r[i][size_t(lk) * m.d + sK];
      if (r < 0 || rk < 0) continue;
      const double sign = (parity && (__builtin_popcount(unsigned(s)) & 1)) ? -1.0 : 1.0;
      const int ml = m.dim[i][l], mlk = m.dim[i][lk], mr = m.dim[i + 1][r], mrk = m.dim[i + 1][rk];
      const double *A = m.data + m.blk_off[i][size_t(l) * m.d + s];     // ml x mr
      const double *B = m.data + m.blk_off[i][size_t(lk) * m.d + sK];   // mlk x mrk
      const std::vector<double> &Xl = X.mat[l];                          // ml x mlk
      tmp.assign(size_t(ml) * mrk, 0.0);                                 // X B
      for (int a = 0; a < ml; ++a)
        for (int b = 0; b < mlk; ++b) {
          const double x = Xl[size_t(a) * mlk + b];
          if (x == 0.0) continue;
          const double *Br = B + size_t(b) * mrk;
          double *T = tmp.data() + size_t(a) * mrk;
          for (int c = 0; c < mrk; ++c) T[c] += x * Br[c];
        }
      if (out.ket[r] < 0) {
        out.ket[r] = rk;
        out.mat[r].assign(size_t(mr) * mrk, 0.0);
      } else if (out.ket[r] != rk) {
        throw std::logic_error("operator sector shift is not fixed");
      }
      double *O = out.mat[r].data();
      for (int a = 0; a < ml; ++a) {
        const double *Ar = A + size_t(a) * mr;
        const double *T = tmp.data() + size_t(a) * mrk;
        for (int r1 = 0; r1 < mr; ++r1) {
          const double x = sign * Ar[r1];
          if (x == 0.0) continue;
          double *Orow = O + size_t(r1) * mrk;
          for (int c = 0; c < mrk; ++c) Orow[c] += x * T[c];
        }
      }
    }
  }
  return out;
}

// Y' = sum_s A^s Y A^{s T} over site i (right environments; identity form).
Op apply_site_right(const Mps &m, int i, const Op &Y) {
  const int nl = int(m.qn[i].size());
  Op out;
  out.ket.assign(nl, -1);
  out.mat.resize(nl);
  std::vector<double> tmp;
  for (int l = 0; l < nl; ++l)
    for (int s = 0; s < m.d; ++s) {
      const int r = m.blk_r[i][size_t(l) * m.d + s];
      if (r < 0 || Y.ket[r] != r) continue;  // identity environments are sector-diagonal
      const int ml = m.dim[i][l], mr = m.dim[i + 1][r];
      const double *A = m.data + m.blk_off[i][size_t(l) * m.d + s];  // ml x mr
      const std::vector<double> &Yr = Y.mat[r];                       // mr x mr
      tmp.assign(size_t(ml) * mr, 0.0);                               // A Y
      for (int a = 0; a < ml; ++a)
        for (int b = 0; b < mr; ++b) {
          const double x = A[size_t(a) * mr + b];
          if (x == 0.0) continue;
          for (int c = 0; c < mr; ++c) tmp[size_t(a) * mr + c] += x * Yr[size_t(b) * mr + c];
        }
      if (out.ket[l] < 0) {
        out.ket[l] = l;
        out.mat[l].assign(size_t(ml) * ml, 0.0);
      }
      double *O = out.mat[l].data();
      for (int a = 0; a < ml; ++a)
        for (int b = 0; b < ml; ++b) {
          double acc = 0.0;
          for (int c = 0; c < mr; ++c) acc += tmp[size_t(a) * mr + c] * A[size_t(b) * mr + c];
          O[size_t(a) * ml + b] += acc;
        }
    }
  return out;
}

// sum_{r,r'} X[r][r'] E[r][r'] over the bra sectors where both map to the
// same ket sector.
double frob(const Op &X, const Op &E) {
  double acc = 0.0;
  for (size_t r = 0; r < X.ket.size(); ++r) {
    if (X.ket[r] < 0 || X.ket[r] != E.ket[r]) continue;
    const auto &a = X.mat[r], &b = E.mat[r];
    for (size_t k = 0; k < a.size(); ++k) acc += a[k] * b[k];
  }
  return acc;
}

// W = A^e E A^{e2 T} at bond j (E the sector-diagonal right environment of
// bond j+1): closing an operator Y of bond j with the pair (e, e2) at site
// j is frob(Y, W).
Op close_op(const Mps &m, int j, int e, int e2, const Op &E) {
  const int nl = int(m.qn[j].size());
  Op out;
  out.ket.assign(nl, -1);
  out.mat.resize(nl);
  std::vector<double> tmp;
  for (int l = 0; l < nl; ++l) {
    const int r = m.blk_r[j][size_t(l) * m.d + e];
    if (r < 0 || E.ket[r] != r) continue;
    const auto qe2 = m.q(e2);
    const int lk = m.find(j, {m.qn[j + 1][r][0] - qe2[0], m.qn[j + 1][r][1] - qe2[1]});
    if (lk < 0) continue;
    const int ml = m.dim[j][l], mlk = m.dim[j][lk], mr = m.dim[j + 1][r];
    const double *A = m.data + m.blk_off[j][size_t(l) * m.d + e];     // ml x mr
    const double *B = m.data + m.blk_off[j][size_t(lk) * m.d + e2];   // mlk x mr
    const std::vector<double> &Er = E.mat[r];                          // mr x mr
    tmp.assign(size_t(ml) * mr, 0.0);                                  // A E
    for (int a = 0; a < ml; ++a)
      for (int b = 0; b < mr; ++b) {
        const double x = A[size_t(a) * mr + b];
        if (x == 0.0) continue;
        for (int c = 0; c < mr; ++c) tmp[size_t(a) * mr + c] += x * Er[size_t(b) * mr + c];
      }
    out.ket[l] = lk;
    out.mat[l].assign(size_t(ml) * mlk, 0.0);
    for (int a = 0; a < ml; ++a)
      for (int b = 0; b < mlk; ++b) {
        double acc = 0.0;
        for (int c = 0; c < mr; ++c) acc += tmp[size_t(a) * mr + c] * B[size_t(b) * mr + c];
        out.mat[l][size_t(a) * mlk + b] = acc;
      }
  }
  return out;
}

// Cyclic Jacobi eigen-decomposition of a symmetric n x n matrix (row-major):
// eigenvalues ascending in w, eigenvectors as the columns of V when wanted.
void jacobi(int n, std::vector<double> A, std::vector<double> &w, std::vector<double> *V) {
  if (V) {
    V->assign(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) (*V)[size_t(i) * n + i] = 1.0;
  }
  double norm = 0.0;
  for (double x : A) norm += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[size_t(p) * n + q] * A[size_t(p) * n + q];
    if (off <= 1e-32 * norm || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = A[size_t(p) * n + q];
        if (apq == 0.0) continue;
        const double app = A[size_t(p) * n + p], aqq = A[size_t(q) * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = A[size_t(k) * n + p], akq = A[size_t(k) * n + q];
          A[size_t(k) * n + p] = c * akp - s * akq;
          A[size_t(k) * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = A[size_t(p) * n + k], aqk = A[size_t(q) * n + k];
          A[size_t(p) * n + k] = c * apk - s * aqk;
          A[size_t(q) * n + k] = s * apk + c * aqk;
        }
        if (V)
          for (int k = 0; k < n; ++k) {
            double *Vr = V->data() + size_t(k) * n;
            const double vkp = Vr[p], vkq = Vr[q];
            Vr[p] = c * vkp - s * vkq;
            Vr[q] = s * vkp + c * vkq;
          }
      }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int a, int b) { return A[size_t(a) * n + a] < A[size_t(b) * n + b]; });
  w.resize(n);
  for (int k = 0; k < n; ++k) w[k] = A[size_t(idx[k]) * n + idx[k]];
  if (V) {
    std::vector<double> W(size_t(n) * n);
    for (int r = 0; r < n; ++r)
      for (int k = 0; k < n; ++k) W[size_t(r) * n + k] = (*V)[size_t(r) * n + idx[k]];
    *V = std::move(W);
  }
}

double vn_entropy(int n, const std::vector<double> &rho) {
  std::vector<double> S(rho);
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b) {
      const double x = 0.5 * (S[size_t(a) * n + b] + S[size_t(b) * n + a]);
      S[size_t(a) * n + b] = S[size_t(b) * n + a] = x;
    }
  std::vector<double> w;
  jacobi(n, S, w, nullptr);
  double s = 0.0;
  for (double x : w)
    if (x > 1e-300) s -= x * std::log(x);
  return s;
}

// <a+_p a_q> on the local Fock space of k spin-orbitals (bit t of a local
// configuration = spin-orbital t, creation operators in bit order):
// matrix element <out|a+_p a_q|in> as (out, sign) or out = -1.
int hop_local(int in, int p, int q, double &sign) {
  if (!((in >> q) & 1)) return -1;
  sign = (__builtin_popcount(unsigned(in) & ((1u << q) - 1u)) & 1) ? -1.0 : 1.0;
  int mid = in ^ (1 << q);
  if ((mid >> p) & 1) return -1;
  if (__builtin_popcount(unsigned(mid) & ((1u << p) - 1u)) & 1) sign = -sign;
  return mid | (1 << p);
}

// Host threads for the analysis: OMP_NUM_THREADS when set, else the
// hardware threads, at most 64.
int host_threads() {
  int nt = int(std::thread::hardware_concurrency());
  if (const char *env = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(env);
    if (v > 0) nt = v;
  }
  return std::max(1, std::min(nt, 64));
}

// Runs task(0..n-1) on host_threads() threads; rethrows the first exception
// a task raised.
template <class F>
void run_parallel(int n, F &&task) {
  const int nt = std::max(1, std::min(n, host_threads()));
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto worker = [&] {
    for (int k; (k = next.fetch_add(1)) < n;) {
      try {
        task(k);
      } catch (...) {
        std::lock_guard<std::mutex> g(mu);
        if (!err) err = std::current_exception();
        next.store(n);
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto &t : pool) t.join();
  if (err) std::rethrow_exception(err);
}

template <class F>
int guarded_host(F &&f) {
  try {
    mdmrg::g_err.clear();
    return f();
  } catch (const std::bad_alloc &) {
    mdmrg::g_err = "host allocation failed";
    return MDMRG_ENOMEM;
  } catch (const std::exception &e) {
    mdmrg::g_err = e.what();
    return MDMRG_EINVAL;
  }
}


// Singular values of the m x n matrix whose n columns are the contiguous
// length-m vectors of X (overwritten), n <= m: one-sided Jacobi (Hestenes)
// -- pairs of columns are rotated until all are mutually orthogonal; the
// singular values are then the column norms, small ones to full accuracy.
std::vector<double> singular_values(int m, int n, std::vector<double> &X) {
  auto col = [&](int j) { return X.data() + size_t(j) * m; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double *xp = col(p), *xq = col(q);
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = 0; i < m; ++i) {
          a += xp[i] * xp[i];
          b += xq[i] * xq[i];
          g += xp[i] * xq[i];
        }
        if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < m; ++i) {
          const double u = xp[i], v = xq[i];
          xp[i] = c * u - sn * v;
          xq[i] = sn * u + c * v;
        }
      }
    if (!rotated) break;
  }
  std::vector<double> sv(n);
  for (int j = 0; j < n; ++j) {
    double a = 0.0;
    for (int i = 0; i < m; ++i) a += col(j)[i] * col(j)[i];
    sv[j] = std::sqrt(a);
  }
  return sv;
}

// Generator of the two-mode rotation on the local space of two adjacent
// sites (bits 0..ns-1 the first site's spin-orbitals, ns..2ns-1 the
// second's): K0 = sum_sigma (a+_{1 sigma} a_{2 sigma} - a+_{2 sigma} a_{1 sigma}),
// and U = exp(theta K0) by scaling and squaring of its Taylor series.
std::vector<double> two_mode_unitary(int ns, double theta) {
  const int D = 1 << (2 * ns);
  std::vector<double> K(size_t(D) * D, 0.0);
  for (int sg = 0; sg < ns; ++sg)
    for (int t = 0; t < D; ++t) {
      double sign;
      int o = hop_local(t, sg, ns + sg, sign);
      if (o >= 0) K[size_t(o) * D + t] += theta * sign;
      o = hop_local(t, ns + sg, sg, sign);
      if (o >= 0) K[size_t(o) * D + t] -= theta * sign;
    }
  int sq = 0;
  double nrm = std::fabs(theta) * 2.0 * ns;
  while (nrm > 0.25) {
    nrm *= 0.5;
    ++sq;
  }
  const double f = std::ldexp(1.0, -sq);
  for (double &x : K) x *= f;
  std::vector<double> U(size_t(D) * D, 0.0), term(size_t(D) * D, 0.0), nxt(size_t(D) * D);
  for (int i = 0; i < D; ++i) U[size_t(i) * D + i] = term[size_t(i) * D + i] = 1.0;
  for (int k = 1; k <= 24; ++k) {
    std::fill(nxt.begin(), nxt.end(), 0.0);
    for (int i = 0; i < D; ++i)
      for (int l = 0; l < D; ++l) {
        const double x = K[size_t(i) * D + l];
        if (x == 0.0) continue;
        for (int j = 0; j < D; ++j) nxt[size_t(i) * D + j] += x * term[size_t(l) * D + j] / k;
      }
    term.swap(nxt);
    for (size_t q = 0; q < U.size(); ++q) U[q] += term[q];
  }
  for (int r = 0; r < sq; ++r) {
    std::fill(nxt.begin(), nxt.end(), 0.0);
    for (int i = 0; i < D; ++i)
      for (int l = 0; l < D; ++l) {
        const double x = U[size_t(i) * D + l];
        if (x == 0.0) continue;
        for (int j = 0; j < D; ++j) nxt[size_t(i) * D + j] += x * U[size_t(l) * D + j];
      }
    U.swap(nxt);
  }
  return U;
}

// The two-site wave function of a bond as blocks (a, s1, s2, b) of
// m_a x m_b doubles (row-major) at given offsets.
struct TwoSite {
  int ns = 1, d = 2, nblk = 0;
  std::vector<std::array<int, 6>> blk;  // a, s1, s2, b, m_a, m_b
  std::vector<int64_t> off;
  // per (a, b): the block index of every local pair t = s1 + d*s2 (-1: none)
  std::vector<std::pair<std::pair<int, int>, std::vector<int>>> ab;
  // bipartition components: rows (a, s1), columns (s2, b)
  std::vector<std::vector<int>> comp_blocks;
};

void parse_two_site(TwoSite &w, int spin_half, int n_blk, const int32_t *desc, int64_t n_elem) {
  w.ns = spin_half ? 2 : 1;
  w.d = 1 << w.ns;
  w.nblk = n_blk;
  std::vector<std::pair<std::pair<int, int>, std::pair<int, int>>> keys;  // ((a,b),(t,k))
  for (int k = 0; k < n_blk; ++k) {
    const int32_t *q = desc + 8 * size_t(k);
    const int64_t off = int64_t(uint32_t(q[6])) | (int64_t(q[7]) << 32);
    if (q[0] < 0 || q[3] < 0 || q[1] < 0 || q[1] >= w.d || q[2] < 0 || q[2] >= w.d || q[4] < 1 || q[5] < 1 ||
        off < 0 || off + int64_t(q[4]) * q[5] > n_elem)
      throw BadInput("a block descriptor is out of range");
    w.blk.push_back({q[0], q[1], q[2], q[3], q[4], q[5]});
    w.off.push_back(off);
    keys.push_back({{q[0], q[3]}, {q[1] + w.d * q[2], k}});
  }
  // every block of a left sector a has the same row count, every block of
  // a right sector b the same column count
  std::vector<std::pair<int, int>> ra, cb;
  for (auto &b : w.blk) {
    ra.push_back({b[0], b[4]});
    cb.push_back({b[3], b[5]});
  }
  for (auto *v : {&ra, &cb}) {
    std::sort(v->begin(), v->end());
    for (size_t k = 1; k < v->size(); ++k)
      if ((*v)[k].first == (*v)[k - 1].first && (*v)[k].second != (*v)[k - 1].second)
        throw BadInput("blocks of one sector disagree on its dimension");
  }
  std::sort(keys.begin(), keys.end());
  for (size_t k = 0; k < keys.size(); ++k) {
    if (k > 0 && keys[k].first == keys[k - 1].first && keys[k].second.first == keys[k - 1].second.first)
      throw BadInput("two blocks share (a, s1, s2, b)");
    if (w.ab.empty() || w.ab.back().first != keys[k].first)
      w.ab.push_back({keys[k].first, std::vector<int>(size_t(w.d) * w.d, -1)});
    w.ab.back().second[keys[k].second.first] = keys[k].second.second;
  }
  // union-find over rows (a, s1) and columns (s2, b) joined by blocks
  std::vector<std::pair<int, int>> rows, cols;
  for (auto &b : w.blk) {
    rows.push_back({b[0], b[1]});
    cols.push_back({b[2], b[3]});
  }
  std::sort(rows.begin(), rows.end());
  rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
  std::sort(cols.begin(), cols.end());
  cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  std::vector<int> parent(rows.size() + cols.size());
  std::iota(parent.begin(), parent.end(), 0);
  std::function<int(int)> root = [&](int x) { return parent[x] == x ? x : parent[x] = root(parent[x]); };
  std::vector<int> brow(n_blk);
  for (int k = 0; k < n_blk; ++k) {
    const auto &b = w.blk[k];
    const int r = int(std::lower_bound(rows.begin(), rows.end(), std::make_pair(b[0], b[1])) - rows.begin());
    const int c = int(std::lower_bound(cols.begin(), cols.end(), std::make_pair(b[2], b[3])) - cols.begin());
    brow[k] = r;
    parent[root(r)] = root(int(rows.size()) + c);
  }
  std::vector<int> label(parent.size(), -1);
  for (int k = 0; k < n_blk; ++k) {
    const int r = root(brow[k]);
    if (label[r] < 0) {
      label[r] = int(w.comp_blocks.size());
      w.comp_blocks.emplace_back();
    }
    w.comp_blocks[label[r]].push_back(k);
  }
}

// psi' = (U (x) 1) psi on the local pair of every (a, b).
void rotate_two_site(const TwoSite &w, const std::vector<double> &U, const double *psi, double *out) {
  const int D = w.d * w.d;
  for (const auto &e : w.ab) {
    const auto &idx = e.second;
    for (int t2 = 0; t2 < D; ++t2) {
      const int k2 = idx[t2];
      if (k2 < 0) continue;
      const int64_t sz = int64_t(w.blk[k2][4]) * w.blk[k2][5];
      double *o = out + w.off[k2];
      std::fill(o, o + sz, 0.0);
      for (int t = 0; t < D; ++t) {
        const double u = U[size_t(t2) * D + t];
        if (u == 0.0) continue;
        const int k = idx[t];
        if (k < 0) throw BadInput("the layout is not closed under the rotation");
        const double *x = psi + w.off[k];
        for (int64_t q = 0; q < sz; ++q) o[q] += u * x[q];
      }
    }
  }
}

// S_1/2 = 2 ln sum_k sqrt(p_k) of the bipartition (a, s1 | s2, b), p_k the
// squared singular values (Schmidt weights) normalised to sum 1.
// The sectors run on the host's threads when `threads` is set.
double half_renyi_two_site(const TwoSite &w, const double *psi, bool threads) {
  const int nc = int(w.comp_blocks.size());
  std::vector<double> part_s(nc, 0.0), part_s2(nc, 0.0);
  auto sector = [&](int ic) {
    const auto &cb = w.comp_blocks[ic];
    // rows (a, s1) and columns (s2, b) of this component
    std::vector<std::pair<int, int>> rows, cols;
    for (int k : cb) {
      rows.push_back({w.blk[k][0], w.blk[k][1]});
      cols.push_back({w.blk[k][2], w.blk[k][3]});
    }
    std::sort(rows.begin(), rows.end());
    rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    auto row_of = [&](int k) {
      return int(std::lower_bound(rows.begin(), rows.end(), std::make_pair(w.blk[k][0], w.blk[k][1])) - rows.begin());
    };
    auto col_of = [&](int k) {
      return int(std::lower_bound(cols.begin(), cols.end(), std::make_pair(w.blk[k][2], w.blk[k][3])) - cols.begin());
    };
    std::vector<int> roff(rows.size() + 1, 0), coff(cols.size() + 1, 0), rdim(rows.size()), cdim(cols.size());
    for (int k : cb) {
      rdim[row_of(k)] = w.blk[k][4];
      cdim[col_of(k)] = w.blk[k][5];
    }
    for (size_t r = 0; r < rows.size(); ++r) roff[r + 1] = roff[r] + rdim[r];
    for (size_t c = 0; c < cols.size(); ++c) coff[c + 1] = coff[c] + cdim[c];
    const int R = roff.back(), C = coff.back();
    // the component matrix with its shorter side as the column count: X holds
    // min(R, C) contiguous vectors of length max(R, C)
    const bool cols_short = C <= R;
    const int m = cols_short ? R : C, n = cols_short ? C : R;
    std::vector<double> X(size_t(m) * n, 0.0);
    for (int k : cb) {
      const int r0 = roff[row_of(k)], c0 = coff[col_of(k)];
      const int ma = w.blk[k][4], mb = w.blk[k][5];
      const double *x = psi + w.off[k];
      for (int i = 0; i < ma; ++i)
        for (int j = 0; j < mb; ++j) {
          const double v = x[size_t(i) * mb + j];
          if (cols_short) X[size_t(c0 + j) * m + r0 + i] = v;
          else X[size_t(r0 + i) * m + c0 + j] = v;
        }
    }
    for (double sv : singular_values(m, n, X)) {
      part_s[ic] += sv;
      part_s2[ic] += sv * sv;
    }
  };
  if (threads) {
    run_parallel(nc, sector);
  } else {
    for (int ic = 0; ic < nc; ++ic) sector(ic);
  }
  double sum_s = 0.0, sum_s2 = 0.0;
  for (int ic = 0; ic < nc; ++ic) {
    sum_s += part_s[ic];
    sum_s2 += part_s2[ic];
  }
  if (!(sum_s2 > 0.0)) throw BadInput("the wave function is zero");
  return 2.0 * std::log(sum_s / std::sqrt(sum_s2));
}

// Exchange arrays of the state whose sites l and l+1 are replaced by the
// two-site wave function psi at bond l (blocks (a, s1, s2, b) over the
// sectors of bonds l and l+2).  It is factored exactly, without an SVD, as
// psi = M * 1: bond l+1 gets one sector per middle quantum number
// Q = Q_a + q(s1), of dimension C_Q = sum of m_b over the (s2, b) with
// Q_b = Q + q(s2); site l holds the rows of M (block (a, s1, Q): psi's
// blocks side by side in (s2, b) order) and site l+1 the identity slices
// (block (Q, s2, b): C_Q x m_b with ones on the columns of (s2, b)).
void merge_centre(const Mps &m, int l, const TwoSite &w, const double *psi, std::vector<int32_t> &n_sect,
                  std::vector<int32_t> &sqn, std::vector<int32_t> &sdim, std::vector<double> &data) {
  const int d = m.d;
  if (l < 0 || l + 2 > m.n) throw BadInput("the centre bond is not a bond of two sites");
  // the blocks of psi by (a, s1, s2, b), checked against the sector lists
  std::vector<int> blk_at(size_t(m.qn[l].size()) * d * d * m.qn[l + 2].size(), -1);
  auto key = [&](int a, int s1, int s2, int b) { return ((size_t(a) * d + s1) * d + s2) * m.qn[l + 2].size() + b; };
  for (int k = 0; k < w.nblk; ++k) {
    const auto &b = w.blk[k];
    if (b[0] >= int(m.qn[l].size()) || b[3] >= int(m.qn[l + 2].size()) || b[4] != m.dim[l][b[0]] ||
        b[5] != m.dim[l + 2][b[3]])
      throw BadInput("a centre block does not match the sectors of its bonds");
    const auto q1 = m.q(b[1]), q2 = m.q(b[2]);
    const auto &Qa = m.qn[l][b[0]], &Qb = m.qn[l + 2][b[3]];
    if (Qa[0] + q1[0] + q2[0] != Qb[0] || Qa[1] + q1[1] + q2[1] != Qb[1])
      throw BadInput("a centre block breaks the quantum-number rule");
    blk_at[key(b[0], b[1], b[2], b[3])] = k;
  }
  // middle sectors and their column layout
  std::vector<std::array<int, 2>> mids;
  for (size_t a = 0; a < m.qn[l].size(); ++a)
    for (int s1 = 0; s1 < d; ++s1) {
      const auto q1 = m.q(s1);
      mids.push_back({m.qn[l][a][0] + q1[0], m.qn[l][a][1] + q1[1]});
    }
  std::sort(mids.begin(), mids.end());
  mids.erase(std::unique(mids.begin(), mids.end()), mids.end());
  std::vector<std::array<int, 2>> qmid;
  std::vector<std::vector<std::array<int, 3>>> colmap;  // per middle sector: (s2, b, column offset)
  std::vector<int> cdim;
  for (const auto &Q : mids) {
    std::vector<std::array<int, 3>> cols;
    int c = 0;
    for (int s2 = 0; s2 < d; ++s2) {
      const auto q2 = m.q(s2);
      const int b = m.find(l + 2, {Q[0] + q2[0], Q[1] + q2[1]});
      if (b < 0) continue;
      cols.push_back({s2, b, c});
      c += m.dim[l + 2][b];
    }
    if (c == 0) continue;
    qmid.push_back(Q);
    colmap.push_back(cols);
    cdim.push_back(c);
  }
  if (qmid.empty()) throw BadInput("the centre has no middle sector");
  // sector lists
  n_sect.clear();
  sqn.clear();
  sdim.clear();
  for (int b = 0; b <= m.n; ++b) {
    if (b == l + 1) {
      n_sect.push_back(int32_t(qmid.size()));
      for (size_t t = 0; t < qmid.size(); ++t) {
        sqn.push_back(qmid[t][0]);
        sqn.push_back(qmid[t][1]);
        sdim.push_back(cdim[t]);
      }
    } else {
      n_sect.push_back(int32_t(m.qn[b].size()));
      for (size_t t = 0; t < m.qn[b].size(); ++t) {
        sqn.push_back(m.qn[b][t][0]);
        sqn.push_back(m.qn[b][t][1]);
        sdim.push_back(m.dim[b][t]);
      }
    }
  }
  // site data: sites < l, the two new sites, sites > l+1
  data.assign(m.data + m.site_off[0], m.data + m.site_off[l]);
  for (size_t a = 0; a < m.qn[l].size(); ++a)
    for (int s1 = 0; s1 < d; ++s1) {
      const auto q1 = m.q(s1);
      const std::array<int, 2> Q{m.qn[l][a][0] + q1[0], m.qn[l][a][1] + q1[1]};
      const auto it = std::lower_bound(qmid.begin(), qmid.end(), Q);
      if (it == qmid.end() || *it != Q) continue;
      const size_t t = size_t(it - qmid.begin());
      const int ma = m.dim[l][a], C = cdim[t];
      const size_t base = data.size();
      data.resize(base + size_t(ma) * C, 0.0);
      for (const auto &cm : colmap[t]) {
        const int k = blk_at[key(int(a), s1, cm[0], cm[1])];
        if (k < 0) continue;  // absent block: zero
        const int mb = m.dim[l + 2][cm[1]];
        const double *x = psi + w.off[k];
        for (int i = 0; i < ma; ++i)
          for (int j = 0; j < mb; ++j) data[base + size_t(i) * C + cm[2] + j] = x[size_t(i) * mb + j];
      }
    }
  for (size_t t = 0; t < qmid.size(); ++t)
    for (int s2 = 0; s2 < d; ++s2)
      for (const auto &cm : colmap[t]) {
        if (cm[0] != s2) continue;
        const int mb = m.dim[l + 2][cm[1]], C = cdim[t];
        const size_t base = data.size();
        data.resize(base + size_t(C) * mb, 0.0);
        for (int j = 0; j < mb; ++j) data[base + size_t(cm[2] + j) * mb + j] = 1.0;
      }
  data.insert(data.end(), m.data + m.site_off[l + 2], m.data + m.site_off[m.n]);
}


// Angles to search: the given ones, else 64 covering [-pi/2, pi/2).
std::vector<double> angle_grid(int n_theta, const double *theta) {
  std::vector<double> grid;
  if (n_theta > 0) {
    grid.assign(theta, theta + n_theta);
  } else {
    for (int k = 0; k < 64; ++k) grid.push_back(-0.5 * M_PI + M_PI * k / 64.0);
  }
  return grid;
}

// The two-mode micro-iteration on a two-site vector: S_1/2 on the grid (one
// angle per thread), then golden-section search within one grid step of the
// best grid angle (sectors on the threads).
void best_angle(const TwoSite &w, const double *psi, int64_t n_elem, const std::vector<double> &grid,
                double *s_grid, double *theta_best, double *s_best) {
  std::vector<double> buf(n_elem, 0.0);
  auto eval = [&](double th) {
    rotate_two_site(w, two_mode_unitary(w.ns, th), psi, buf.data());
    return half_renyi_two_site(w, buf.data(), true);
  };
  std::vector<double> val(grid.size());
  run_parallel(int(grid.size()), [&](int k) {
    std::vector<double> mine(n_elem, 0.0);
    rotate_two_site(w, two_mode_unitary(w.ns, grid[k]), psi, mine.data());
    val[k] = half_renyi_two_site(w, mine.data(), false);
  });
  if (s_grid) std::copy(val.begin(), val.end(), s_grid);
  const size_t kb = size_t(std::min_element(val.begin(), val.end()) - val.begin());
  double best_t = grid[kb], best_v = val[kb];
  double step = 0.0;
  for (size_t k = 1; k < grid.size(); ++k) step = std::max(step, std::fabs(grid[k] - grid[k - 1]));
  if (grid.size() > 1 && step > 0.0) {
    const double g = 0.5 * (std::sqrt(5.0) - 1.0);
    double a = best_t - step, b = best_t + step;
    double x1 = b - g * (b - a), x2 = a + g * (b - a);
    double f1 = eval(x1), f2 = eval(x2);
    for (int it = 0; it < 80 && b - a > 1e-12; ++it) {
      if (f1 < f2) {
        b = x2; x2 = x1; f2 = f1; x1 = b - g * (b - a); f1 = eval(x1);
      } else {
        a = x1; x1 = x2; f1 = f2; x2 = a + g * (b - a); f2 = eval(x2);
      }
    }
    const double xm = f1 < f2 ? x1 : x2, fm = std::min(f1, f2);
    if (fm < best_v) {
      best_v = fm;
      best_t = xm;
    }
  }
  *theta_best = best_t;
  *s_best = best_v;
}

// Exact factorisation M = L C of an R x Cn matrix (row-major): one-sided
// Jacobi on the shorter side's vectors.  L (R x r) has orthonormal columns,
// C = S V^T (r x Cn); singular values at or below 1e-15 of the largest are
// dropped (rank r).  Returns r.
int factor_lc(int R, int Cn, const std::vector<double> &M, std::vector<double> &L, std::vector<double> &C) {
  const bool cols_short = Cn <= R;
  const int m = cols_short ? R : Cn, n = cols_short ? Cn : R;
  std::vector<double> X(size_t(m) * n), J(size_t(n) * n, 0.0);
  for (int i = 0; i < R; ++i)
    for (int j = 0; j < Cn; ++j) {
      if (cols_short) X[size_t(j) * m + i] = M[size_t(i) * Cn + j];
      else X[size_t(i) * m + j] = M[size_t(i) * Cn + j];
    }
  for (int i = 0; i < n; ++i) J[size_t(i) * n + i] = 1.0;  // J[col q][row p]: vector q of J
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double *xp = X.data() + size_t(p) * m, *xq = X.data() + size_t(q) * m;
        double a = 0.0, b = 0.0, g = 0.0;
        for (int i = 0; i < m; ++i) {
          a += xp[i] * xp[i];
          b += xq[i] * xq[i];
          g += xp[i] * xq[i];
        }
        if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = c * t;
        for (int i = 0; i < m; ++i) {
          const double u = xp[i], v = xq[i];
          xp[i] = c * u - sn * v;
          xq[i] = sn * u + c * v;
        }
        double *jp = J.data() + size_t(p) * n, *jq = J.data() + size_t(q) * n;
        for (int i = 0; i < n; ++i) {
          const double u = jp[i], v = jq[i];
          jp[i] = c * u - sn * v;
          jq[i] = sn * u + c * v;
        }
      }
    if (!rotated) break;
  }
  // X_q = (A J)_q with A the matrix whose columns were rotated; sigma_q = |X_q|
  std::vector<double> sig(n);
  double smax = 0.0;
  for (int q = 0; q < n; ++q) {
    double a = 0.0;
    for (int i = 0; i < m; ++i) a += X[size_t(q) * m + i] * X[size_t(q) * m + i];
    sig[q] = std::sqrt(a);
    smax = std::max(smax, sig[q]);
  }
  std::vector<int> keep;
  for (int q = 0; q < n; ++q)
    if (sig[q] > 1e-15 * smax && sig[q] > 0.0) keep.push_back(q);
  const int r = int(keep.size());
  L.assign(size_t(R) * r, 0.0);
  C.assign(size_t(r) * Cn, 0.0);
  for (int t = 0; t < r; ++t) {
    const int q = keep[t];
    if (cols_short) {
      // M J = X (R x n): M = X J^T; L = X_q / sigma_q, C row t = sigma_q J_q^T
      for (int i = 0; i < R; ++i) L[size_t(i) * r + t] = X[size_t(q) * m + i] / sig[q];
      for (int j = 0; j < Cn; ++j) C[size_t(t) * Cn + j] = sig[q] * J[size_t(q) * n + j];
    } else {
      // M^T J = X (Cn x n): M = J X^T; L column t = J_q, C row t = X_q^T
      for (int i = 0; i < R; ++i) L[size_t(i) * r + t] = J[size_t(q) * n + i];
      for (int j = 0; j < Cn; ++j) C[size_t(t) * Cn + j] = X[size_t(q) * m + j];
    }
  }
  return r;
}

}  // namespace

extern "C" {

int mdmrg_mode_analysis(int n_sites, int spin_half, const int32_t *n_sect, const int32_t *sect_qn,
                        const int32_t *sect_dim, const double *data, int64_t n_data, double *s_one,
                        double *s_two, double *rho_one, double *rho_two, double *gamma, double *occ,
                        double *nn, int centre, int n_blk, const int32_t *desc, const double *psi,
                        int64_t n_psi) {
  if (n_sites < 1 || !n_sect || !sect_qn || !sect_dim || (!data && n_data > 0) || !s_one || !s_two ||
      (centre >= 0 && (n_blk < 1 || !desc || !psi || n_psi < 1)))
    return MDMRG_EINVAL;
  return guarded_host([&] {
    Mps m;
    parse(m, n_sites, spin_half, n_sect, sect_qn, sect_dim, data, n_data);
    std::vector<int32_t> c_sect, c_qn, c_dim;
    std::vector<double> c_data;
    if (centre >= 0) {  // the state with its two-site centre at bond `centre`
      TwoSite w;
      parse_two_site(w, spin_half, n_blk, desc, n_psi);
      merge_centre(m, centre, w, psi, c_sect, c_qn, c_dim, c_data);
      m = Mps();
      parse(m, n_sites, spin_half, c_sect.data(), c_qn.data(), c_dim.data(), c_data.data(),
            int64_t(c_data.size()));
    }
    const int n = m.n, d = m.d, ns = m.ns, nso = n * ns, d2 = d * d;
    // identity environments and the closing operators of every site
    std::vector<Op> EL(n + 1), ER(n + 1);
    EL[0] = identity_op(m, 0);
    for (int i = 0; i < n; ++i) EL[i + 1] = apply_site(m, i, EL[i], -1, -1, false);
    ER[n] = identity_op(m, n);
    for (int i = n - 1; i >= 0; --i) ER[i] = apply_site_right(m, i, ER[i + 1]);
    const double Z = frob(EL[n], ER[n]);
    if (!(Z > 0.0) || !std::isfinite(Z)) throw BadInput("the state has no norm");
    std::vector<Op> W(size_t(n) * d * d);
    for (int j = 0; j < n; ++j)
      for (int e = 0; e < d; ++e)
        for (int e2 = 0; e2 < d; ++e2) W[(size_t(j) * d + e) * d + e2] = close_op(m, j, e, e2, ER[j + 1]);
    if (gamma) std::fill(gamma, gamma + size_t(nso) * nso, 0.0);

    // one site i per task: rho_i, then rho_ij for every j > i
    auto site_task = [&](int i) {
      std::vector<double> r1(size_t(d) * d);
      for (int c = 0; c < d; ++c)
        for (int c2 = 0; c2 < d; ++c2) r1[size_t(c) * d + c2] = frob(EL[i], W[(size_t(i) * d + c) * d + c2]) / Z;
      s_one[i] = vn_entropy(d, r1);
      s_two[size_t(i) * n + i] = s_one[i];
      if (rho_one) std::copy(r1.begin(), r1.end(), rho_one + size_t(i) * d * d);
      if (occ)
        for (int t = 0; t < ns; ++t) {
          double o = 0.0;
          for (int c = 0; c < d; ++c)
            if ((c >> t) & 1) o += r1[size_t(c) * d + c];
          occ[size_t(i) * ns + t] = o;
        }
      if (nn) {  // <n_i^2>, n_i the particle number of the mode
        double o = 0.0;
        for (int c = 0; c < d; ++c) {
          const int nc = __builtin_popcount(unsigned(c));
          o += r1[size_t(c) * d + c] * nc * nc;
        }
        nn[size_t(i) * n + i] = o;
      }
      if (gamma)  // same-site elements <a+_p a_q> = sum_in sign rho[in][out]
        for (int p = 0; p < ns; ++p)
          for (int q = 0; q < ns; ++q) {
            double g = 0.0, sg;
            for (int a = 0; a < d; ++a) {
              const int b = hop_local(a, p, q, sg);
              if (b >= 0) g += sg * r1[size_t(a) * d + b];
            }
            gamma[size_t(i * ns + p) * nso + i * ns + q] = g;
          }
      if (i + 1 >= n) return;
      // blocks of rho_ij for all j > i, local index c + d*e (modes i, j)
      std::vector<double> blks(size_t(n - i - 1) * d2 * d2);
      for (int c = 0; c < d; ++c)
        for (int c2 = 0; c2 < d; ++c2) {
          const bool parity = (__builtin_popcount(unsigned(c)) + __builtin_popcount(unsigned(c2))) & 1;
          Op Y = apply_site(m, i, EL[i], c, c2, false);
          for (int j = i + 1; j < n; ++j) {
            double *blk = blks.data() + size_t(j - i - 1) * d2 * d2;
            for (int e = 0; e < d; ++e)
              for (int e2 = 0; e2 < d; ++e2)
                blk[(size_t(c) + size_t(d) * e) * d2 + size_t(c2) + size_t(d) * e2] =
                    frob(Y, W[(size_t(j) * d + e) * d + e2]) / Z;
            if (j + 1 < n) Y = apply_site(m, j, Y, -1, -1, parity);
          }
        }
      for (int j = i + 1; j < n; ++j) {
        const double *blk = blks.data() + size_t(j - i - 1) * d2 * d2;
        const double sij = vn_entropy(d2, std::vector<double>(blk, blk + size_t(d2) * d2));
        s_two[size_t(i) * n + j] = s_two[size_t(j) * n + i] = sij;
        if (nn) {  // <n_i n_j> from the diagonal of rho_ij
          double o = 0.0;
          for (int c = 0; c < d; ++c)
            for (int e = 0; e < d; ++e) {
              const size_t t = size_t(c) + size_t(d) * e;
              o += blk[t * d2 + t] * __builtin_popcount(unsigned(c)) * __builtin_popcount(unsigned(e));
            }
          nn[size_t(i) * n + j] = nn[size_t(j) * n + i] = o;
        }
        if (rho_two) {
          std::copy(blk, blk + size_t(d2) * d2, rho_two + (size_t(i) * n + j) * d2 * d2);
          // modes listed (j, i): local index e + d*c and the reordering sign
          // (-1)^{N(c)N(e) + N(c')N(e')}
          double *out = rho_two + (size_t(j) * n + i) * d2 * d2;
          for (int c = 0; c < d; ++c)
            for (int e = 0; e < d; ++e)
              for (int c2 = 0; c2 < d; ++c2)
                for (int e2 = 0; e2 < d; ++e2) {
                  const int sg = (__builtin_popcount(unsigned(c)) * __builtin_popcount(unsigned(e)) +
                                  __builtin_popcount(unsigned(c2)) * __builtin_popcount(unsigned(e2))) & 1;
                  const double v = blk[(size_t(c) + size_t(d) * e) * d2 + size_t(c2) + size_t(d) * e2];
                  out[(size_t(e) + size_t(d) * c) * d2 + size_t(e2) + size_t(d) * c2] = sg ? -v : v;
                }
        }
        if (gamma)  // <a+_p a_q> with p and q on different sites of the pair
          for (int p = 0; p < 2 * ns; ++p)
            for (int q = 0; q < 2 * ns; ++q) {
              if ((p < ns) == (q < ns)) continue;
              double g = 0.0, sg;
              for (int a = 0; a < d2; ++a) {
                const int b = hop_local(a, p, q, sg);
                if (b >= 0) g += sg * blk[size_t(a) * d2 + b];
              }
              const int gp = p < ns ? i * ns + p : j * ns + (p - ns);
              const int gq = q < ns ? i * ns + q : j * ns + (q - ns);
              gamma[size_t(gp) * nso + gq] = g;
            }
      }
    };
    run_parallel(n, site_task);
    return MDMRG_OK;
  });
}

int mdmrg_cdw_order(int n, const double *nn, const double *sign, double *c_cdw) {
  if (n < 1 || !nn || !sign || !c_cdw) return MDMRG_EINVAL;
  return guarded_host([&] {
    double num = 0.0, n2 = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        num += sign[i] * sign[j] * nn[size_t(i) * n + j];
        n2 += nn[size_t(i) * n + j];
      }
    if (!(n2 > 0.0)) throw BadInput("the state holds no particles");
    *c_cdw = num / n2;
    return MDMRG_OK;
  });
}

int mdmrg_mutual_information(int n, const double *s_one, const double *s_two, const int32_t *order,
                             double *I, double *i_tot, double *i_dist) {
  if (n < 1 || !s_one || !s_two || !I) return MDMRG_EINVAL;
  return guarded_host([&] {
    std::vector<int> pos(n);
    std::iota(pos.begin(), pos.end(), 0);
    if (order) {
      std::vector<int> seen(n, 0);
      for (int k = 0; k < n; ++k) {
        if (order[k] < 0 || order[k] >= n || seen[order[k]]++) throw BadInput("order is not a permutation");
        pos[order[k]] = k;
      }
    }
    double tot = 0.0, dist = 0.0;
    for (int i = 0; i < n; ++i) {
      tot += s_one[i];
      for (int j = 0; j < n; ++j) {
        const double v = i == j ? 0.0 : s_one[i] + s_one[j] - s_two[size_t(i) * n + j];
        I[size_t(i) * n + j] = v;
        const double dd = double(pos[i] - pos[j]);
        dist += v * dd * dd;
      }
    }
    if (i_tot) *i_tot = tot;
    if (i_dist) *i_dist = dist;
    return MDMRG_OK;
  });
}

int mdmrg_fiedler_order(int n, const double *I, int32_t *order) {
  if (n < 2 || !I || !order) return MDMRG_EINVAL;
  return guarded_host([&] {
    std::vector<double> L(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        if (i == j) continue;
        const double w = 0.5 * (I[size_t(i) * n + j] + I[size_t(j) * n + i]);
        if (!std::isfinite(w)) throw BadInput("non-finite mutual information");
        L[size_t(i) * n + j] = -w;
        L[size_t(i) * n + i] += w;
      }
    std::vector<double> w, V;
    jacobi(n, L, w, &V);
    if (!(w[1] > 1e-12 * std::max(w[n - 1], 1e-300))) throw BadInput("the graph is disconnected");
    std::vector<double> v(n);
    double corr = 0.0;
    for (int i = 0; i < n; ++i) {
      v[i] = V[size_t(i) * n + 1];
      corr += v[i] * (i - 0.5 * (n - 1));
    }
    if (corr < 0)
      for (double &x : v) x = -x;
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return v[a] < v[b]; });
    for (int k = 0; k < n; ++k) order[k] = idx[k];
    return MDMRG_OK;
  });
}

int mdmrg_deas_order(int n, const double *s_one, int32_t *order) {
  if (n < 1 || !s_one || !order) return MDMRG_EINVAL;
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return s_one[a] > s_one[b]; });
  for (int k = 0; k < n; ++k) order[k] = idx[k];
  return MDMRG_OK;
}

int mdmrg_hf_reference(int n_sites, int spin_half, const double *occ, int target_a, int target_b,
                       int8_t *config) {
  const int ns = spin_half ? 2 : 1;
  if (n_sites < 1 || !occ || !config || target_a < 0 || target_a > n_sites ||
      (spin_half && (target_b < 0 || target_b > n_sites)))
    return MDMRG_EINVAL;
  std::fill(config, config + size_t(n_sites) * ns, int8_t(0));
  for (int sigma = 0; sigma < ns; ++sigma) {
    const int k = sigma == 0 ? target_a : target_b;
    std::vector<int> so(n_sites);
    for (int i = 0; i < n_sites; ++i) so[i] = i * ns + sigma;
    std::stable_sort(so.begin(), so.end(), [&](int a, int b) { return occ[a] > occ[b]; });
    for (int t = 0; t < k; ++t) config[so[t]] = 1;
  }
  return MDMRG_OK;
}

int mdmrg_natural_orbitals(int nso, const double *gamma, double *occupation, double *modes) {
  if (nso < 1 || !gamma || !occupation) return MDMRG_EINVAL;
  return guarded_host([&] {
    std::vector<double> G(size_t(nso) * nso);
    for (int a = 0; a < nso; ++a)
      for (int b = 0; b < nso; ++b)
        G[size_t(a) * nso + b] = 0.5 * (gamma[size_t(a) * nso + b] + gamma[size_t(b) * nso + a]);
    std::vector<double> w, V;
    jacobi(nso, G, w, modes ? &V : nullptr);
    for (int k = 0; k < nso; ++k) occupation[k] = w[nso - 1 - k];  // descending
    if (modes)
      for (int r = 0; r < nso; ++r)
        for (int k = 0; k < nso; ++k) modes[size_t(r) * nso + k] = V[size_t(r) * nso + nso - 1 - k];
    return MDMRG_OK;
  });
}

int mdmrg_two_mode_rotation(int spin_half, int n_blk, const int32_t *desc, const double *psi, int64_t n_elem,
                            int n_theta, const double *theta, double *s_half, double *theta_best,
                            double *s_best, double *psi_rotated) {
  if (n_blk < 1 || !desc || !psi || n_elem < 1 || n_theta < 0 || (n_theta > 0 && (!theta || !s_half)) ||
      !theta_best || !s_best || psi_rotated == psi)
    return MDMRG_EINVAL;
  return guarded_host([&] {
    TwoSite w;
    parse_two_site(w, spin_half, n_blk, desc, n_elem);
    const std::vector<double> grid = angle_grid(n_theta, theta);
    best_angle(w, psi, n_elem, grid, n_theta > 0 ? s_half : nullptr, theta_best, s_best);
    if (psi_rotated) rotate_two_site(w, two_mode_unitary(w.ns, *theta_best), psi, psi_rotated);
    return MDMRG_OK;
  });
}

int mdmrg_rotation_sweep(int n_sites, int spin_half, const int32_t *n_sect, const int32_t *sect_qn,
                         const int32_t *sect_dim, const double *data, int64_t n_data, int n_blk,
                         const int32_t *desc, const double *psi, int64_t n_psi, int n_theta,
                         const double *theta_grid, double *theta, double *s_half, double *R) {
  if (n_sites < 2 || !n_sect || !sect_qn || !sect_dim || (!data && n_data > 0) || n_blk < 1 || !desc || !psi ||
      n_psi < 1 || n_theta < 0 || (n_theta > 0 && !theta_grid) || !theta || !s_half || !R)
    return MDMRG_EINVAL;
  return guarded_host([&] {
    Mps m;
    parse(m, n_sites, spin_half, n_sect, sect_qn, sect_dim, data, n_data);
    const int n = m.n, d = m.d;
    const std::vector<double> grid = angle_grid(n_theta, theta_grid);
    // the centre at bond k: sectors of bond k (left) and k+2 (right), blocks
    // for every (a, s1, s2, b) of the sector rule, packed in that order
    std::vector<std::array<int, 2>> lq(m.qn[0]);
    std::vector<int> ld(m.dim[0]);
    std::vector<int32_t> cdesc;
    std::vector<double> cpsi;
    auto layout = [&](int k) {  // cdesc for the current left sectors, bond k+2 on the right
      cdesc.clear();
      int64_t off = 0;
      for (size_t a = 0; a < lq.size(); ++a)
        for (int s1 = 0; s1 < d; ++s1)
          for (int s2 = 0; s2 < d; ++s2) {
            const auto q1 = m.q(s1), q2 = m.q(s2);
            const int b = m.find(k + 2, {lq[a][0] + q1[0] + q2[0], lq[a][1] + q1[1] + q2[1]});
            if (b < 0) continue;
            const int mb = m.dim[k + 2][b];
            const int32_t v[8] = {int32_t(a), s1, s2, b, ld[a], mb, int32_t(off & 0xFFFFFFFF), int32_t(off >> 32)};
            cdesc.insert(cdesc.end(), v, v + 8);
            off += int64_t(ld[a]) * mb;
          }
      return off;
    };
    // the given centre, copied into the packed layout of bond 0
    {
      const int64_t ne = layout(0);
      TwoSite w0;
      parse_two_site(w0, spin_half, n_blk, desc, n_psi);
      cpsi.assign(ne, 0.0);
      TwoSite wl;
      parse_two_site(wl, spin_half, int(cdesc.size() / 8), cdesc.data(), ne);
      for (int k = 0; k < w0.nblk; ++k) {
        const auto &b = w0.blk[k];
        if (b[0] >= int(lq.size()) || b[3] >= int(m.qn[2].size()) || b[4] != ld[b[0]] || b[5] != m.dim[2][b[3]])
          throw BadInput("a centre block does not match the sectors of its bonds");
        int found = -1;
        for (int t = 0; t < wl.nblk && found < 0; ++t)
          if (wl.blk[t][0] == b[0] && wl.blk[t][1] == b[1] && wl.blk[t][2] == b[2] && wl.blk[t][3] == b[3]) found = t;
        if (found < 0) throw BadInput("a centre block breaks the quantum-number rule");
        std::copy(psi + w0.off[k], psi + w0.off[k] + int64_t(b[4]) * b[5], cpsi.begin() + wl.off[found]);
      }
    }
    for (int i = 0; i < n * n; ++i) R[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
    for (int k = 0; k + 1 < n; ++k) {
      const int64_t ne = int64_t(cpsi.size());
      TwoSite w;
      parse_two_site(w, spin_half, int(cdesc.size() / 8), cdesc.data(), ne);
      double th, sv;
      best_angle(w, cpsi.data(), ne, grid, nullptr, &th, &sv);
      theta[k] = th;
      s_half[k] = sv;
      std::vector<double> rot(ne, 0.0);
      rotate_two_site(w, two_mode_unitary(w.ns, th), cpsi.data(), rot.data());
      std::map<std::array<int, 4>, int> where;  // (a, s1, s2, b) -> block
      for (int t = 0; t < w.nblk; ++t) where[{w.blk[t][0], w.blk[t][1], w.blk[t][2], w.blk[t][3]}] = t;
      const double c = std::cos(th), sn = std::sin(th);  // R <- R G_k
      for (int r = 0; r < n; ++r) {
        const double x = R[size_t(r) * n + k], y = R[size_t(r) * n + k + 1];
        R[size_t(r) * n + k] = c * x + sn * y;
        R[size_t(r) * n + k + 1] = -sn * x + c * y;
      }
      if (k + 2 >= n) break;
      // move the centre: per middle sector Q, rows (a, s1) | columns (s2, b)
      // factored exactly as L C (L orthonormal columns, C = S V^T), rank kept
      std::vector<std::array<int, 2>> nq;
      std::vector<int> nd;
      std::vector<std::vector<double>> Cq;                   // r x (columns) per new sector
      std::vector<std::vector<std::array<int, 3>>> colsq;    // (s2, b, column offset)
      for (const auto &Q : [&] {
             std::vector<std::array<int, 2>> v;
             for (size_t a = 0; a < lq.size(); ++a)
               for (int s1 = 0; s1 < d; ++s1) v.push_back({lq[a][0] + m.q(s1)[0], lq[a][1] + m.q(s1)[1]});
             std::sort(v.begin(), v.end());
             v.erase(std::unique(v.begin(), v.end()), v.end());
             return v;
           }()) {
        std::vector<std::array<int, 3>> rows, cols;  // (a, s1, row offset), (s2, b, column offset)
        int Rn = 0, Cn = 0;
        for (size_t a = 0; a < lq.size(); ++a)
          for (int s1 = 0; s1 < d; ++s1)
            if (lq[a][0] + m.q(s1)[0] == Q[0] && lq[a][1] + m.q(s1)[1] == Q[1]) {
              rows.push_back({int(a), s1, Rn});
              Rn += ld[a];
            }
        for (int s2 = 0; s2 < d; ++s2) {
          const int b = m.find(k + 2, {Q[0] + m.q(s2)[0], Q[1] + m.q(s2)[1]});
          if (b < 0) continue;
          cols.push_back({s2, b, Cn});
          Cn += m.dim[k + 2][b];
        }
        if (Rn == 0 || Cn == 0) continue;
        std::vector<double> M(size_t(Rn) * Cn, 0.0);
        for (const auto &rw : rows)
          for (const auto &cl : cols) {
            const auto it = where.find({rw[0], rw[1], cl[0], cl[1]});
            if (it == where.end()) continue;
            const auto &bk = w.blk[it->second];
            const double *x = rot.data() + w.off[it->second];
            for (int i = 0; i < bk[4]; ++i)
              for (int j = 0; j < bk[5]; ++j) M[size_t(rw[2] + i) * Cn + cl[2] + j] = x[size_t(i) * bk[5] + j];
          }
        std::vector<double> L, C;
        const int r = factor_lc(Rn, Cn, M, L, C);
        if (r == 0) continue;
        // the new site tensor (L) is not needed for the angles; C carries on
        nq.push_back(Q);
        nd.push_back(r);
        Cq.push_back(std::move(C));
        colsq.push_back(cols);
        (void)L;
      }
      if (nq.empty()) throw BadInput("the state vanished while moving the centre");
      // the next centre: psi'(mid, s2, s3, c) = sum_b C(mid; s2, b) A_{k+2}(b, s3, c)
      lq = nq;
      ld = nd;
      const int64_t ne2 = layout(k + 1);
      cpsi.assign(ne2, 0.0);
      TwoSite wn;
      parse_two_site(wn, spin_half, int(cdesc.size() / 8), cdesc.data(), ne2);
      for (int t = 0; t < wn.nblk; ++t) {
        const auto &bk = wn.blk[t];  // (mid, s2, s3, c)
        const int mid = bk[0], s2 = bk[1], s3 = bk[2], cc = bk[3];
        const int r = nd[mid], mc = bk[5];
        for (const auto &cl : colsq[mid]) {
          if (cl[0] != s2) continue;
          const int b = cl[1];
          if (m.blk_r[k + 2][size_t(b) * d + s3] != cc) continue;
          const int mb = m.dim[k + 2][b];
          const double *A = m.data + m.blk_off[k + 2][size_t(b) * d + s3];  // mb x mc
          const std::vector<double> &Cm = Cq[mid];                          // r x Cn
          const int Cn = int(Cm.size() / size_t(r));
          double *o = cpsi.data() + wn.off[t];
          for (int i = 0; i < r; ++i)
            for (int j = 0; j < mb; ++j) {
              const double x = Cm[size_t(i) * Cn + cl[2] + j];
              if (x == 0.0) continue;
              for (int q = 0; q < mc; ++q) o[size_t(i) * mc + q] += x * A[size_t(j) * mc + q];
            }
        }
      }
    }
    return MDMRG_OK;
  });
}

}  // extern "C"
