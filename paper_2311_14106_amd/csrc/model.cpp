// Model parameters of Eq. (1)-(3) (Sec. II.A), the mode transformation on
// T, V (Sec. II.B), validation, and the canonical operator-term list that the
// engine partitions at every bond.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <thread>
#include <vector>

#include "model.h"

namespace mdmrg {

static int snake(int x, int y, int Lx) { return y * Lx + ((y % 2 == 0) ? x : Lx - 1 - x); }

static void torus_bonds(int Lx, int Ly, std::vector<std::pair<int, int>> &out) {
  out.clear();
  for (int y = 0; y < Ly; ++y)
    for (int x = 0; x < Lx; ++x) {
      const int nb[2][2] = {{(x + 1) % Lx, y}, {x, (y + 1) % Ly}};
      for (auto &q : nb) {
        if (q[0] == x && q[1] == y) continue;  // extent-1 direction: no bond
        out.push_back({snake(x, y, Lx), snake(q[0], q[1], Lx)});
      }
    }
}

int lattice_nso(int model, int Lx, int Ly) { return (model == 1 ? 2 : 1) * Lx * Ly; }

// chain position of every plane-wave mode label m = b*Lx + a, ascending
// eps_k = -2t(cos kx + cos ky), ties by label
static std::vector<int> momentum_positions(int Lx, int Ly, double t, std::vector<double> &eps) {
  const int n = Lx * Ly;
  eps.assign(n, 0.0);
  std::vector<double> key(n);
  for (int m = 0; m < n; ++m) {
    const double kx = 2.0 * M_PI * (m % Lx) / Lx, ky = 2.0 * M_PI * (m / Lx) / Ly;
    eps[m] = -2.0 * t * (std::cos(kx) + std::cos(ky));
    key[m] = std::nearbyint(eps[m] * 1e12) / 1e12;
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] < key[b]; });
  std::vector<int> pos(n);
  for (int c = 0; c < n; ++c) pos[order[c]] = c;
  return pos;
}

void build_lattice(int model, int basis, int Lx, int Ly, double t, double u, double *T, double *V) {
  MDMRG_REQUIRE(Lx >= 1 && Ly >= 1 && (model == 0 || model == 1) && (basis == 0 || basis == 1), -1,
                "build_lattice: bad arguments");
  const int n = Lx * Ly, ns = (model == 1) ? 2 : 1, nso = ns * n;
  const int64_t n2 = int64_t(nso) * nso, n4 = n2 * n2;
  std::fill(T, T + n2, 0.0);
  std::fill(V, V + n4, 0.0);
  auto v4 = [&](int p, int q, int r, int s) -> double & {
    return V[((int64_t(p) * nso + q) * nso + r) * nso + s];
  };
  if (basis == 0) {
    std::vector<std::pair<int, int>> bonds;
    torus_bonds(Lx, Ly, bonds);
    for (auto &b : bonds) {
      for (int s = 0; s < ns; ++s) {
        T[int64_t(ns * b.first + s) * nso + ns * b.second + s] += -t;
        T[int64_t(ns * b.second + s) * nso + ns * b.first + s] += -t;
      }
      if (model == 0) v4(b.first, b.second, b.second, b.first) += u;  // n_i n_j
    }
    if (model == 1)
      for (int i = 0; i < n; ++i) v4(2 * i, 2 * i + 1, 2 * i + 1, 2 * i) += u;  // n_up n_dn
    return;
  }
  std::vector<double> eps;
  std::vector<int> pos = momentum_positions(Lx, Ly, t, eps);
  for (int m = 0; m < n; ++m)
    for (int s = 0; s < ns; ++s) T[int64_t(ns * pos[m] + s) * nso + ns * pos[m] + s] = eps[m];
  for (int m1 = 0; m1 < n; ++m1)
    for (int m2 = 0; m2 < n; ++m2)
      for (int m3 = 0; m3 < n; ++m3) {
        const int a1 = m1 % Lx, b1 = m1 / Lx, a2 = m2 % Lx, b2 = m2 / Lx, a3 = m3 % Lx, b3 = m3 / Lx;
        const int a4 = ((a1 + a2 - a3) % Lx + Lx) % Lx, b4 = ((b1 + b2 - b3) % Ly + Ly) % Ly;
        const int m4 = b4 * Lx + a4;
        if (model == 0) {
          const double qx = 2.0 * M_PI * (a3 - a2) / Lx, qy = 2.0 * M_PI * (b3 - b2) / Ly;
          v4(pos[m1], pos[m2], pos[m3], pos[m4]) += u / n * (std::cos(qx) + std::cos(qy));
        } else {
          v4(2 * pos[m1], 2 * pos[m2] + 1, 2 * pos[m3] + 1, 2 * pos[m4]) += u / n;
        }
      }
}

// Runs f(0..n-1) in contiguous chunks on OMP_NUM_THREADS host threads
// (default: the hardware threads; at most 64).
template <class F>
static void parallel_rows(int64_t n, F &&f) {
  int nt = int(std::thread::hardware_concurrency());
  if (const char *env = std::getenv("OMP_NUM_THREADS")) {
    const int v = std::atoi(env);
    if (v > 0) nt = v;
  }
  nt = int(std::max<int64_t>(1, std::min<int64_t>({int64_t(nt), int64_t(64), n})));
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t] {
      const int64_t lo = n * t / nt, hi = n * (t + 1) / nt;
      for (int64_t k = lo; k < hi; ++k) f(k);
    });
  for (auto &th : pool) th.join();
}

void rotate_modes(int n, int spin_half, const double *R, double *T, double *V) {
  // orthogonality check
  double err = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int a = 0; a < n; ++a) s += R[a * n + i] * R[a * n + j];
      err = std::max(err, std::fabs(s - (i == j ? 1.0 : 0.0)));
    }
  MDMRG_REQUIRE(err < 1e-10, -1, "rotate_modes: R is not orthogonal");
  const int ns = spin_half ? 2 : 1, m = ns * n;
  std::vector<double> Rs(int64_t(m) * m, 0.0);
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i)
      for (int s = 0; s < ns; ++s) Rs[int64_t(ns * a + s) * m + ns * i + s] = R[a * n + i];
  // T <- R^T T R
  std::vector<double> tmp(int64_t(m) * m, 0.0), T2(int64_t(m) * m, 0.0);
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) {
      const double tab = T[int64_t(a) * m + b];
      if (tab == 0.0) continue;
      for (int j = 0; j < m; ++j) tmp[int64_t(a) * m + j] += tab * Rs[int64_t(b) * m + j];
    }
  for (int a = 0; a < m; ++a)
    for (int i = 0; i < m; ++i) {
      const double r = Rs[int64_t(a) * m + i];
      if (r == 0.0) continue;
      for (int j = 0; j < m; ++j) T2[int64_t(i) * m + j] += r * tmp[int64_t(a) * m + j];
    }
  std::copy(T2.begin(), T2.end(), T);
  // V: four one-index transforms.  With V viewed as [alpha, a, beta]
  // (alpha the indices before the transformed one, beta those after),
  // W[alpha, i, :] = sum_a R[a,i] V[alpha, a, :], a ascending: contiguous
  // rows of length m^(3-axis), one (alpha, i) row per work item on the host
  // threads (the last axis, whose rows have length 1, one alpha per item).
  const int64_t m4 = int64_t(m) * m * m * m;
  std::vector<double> W(m4);
  std::vector<char> nz;
  for (int axis = 0; axis < 4; ++axis) {
    int64_t B = 1, A = 1;
    for (int k = 0; k < 3 - axis; ++k) B *= m;
    for (int k = 0; k < axis; ++k) A *= m;
    // rows V[alpha, a, :] that are entirely zero are skipped
    nz.assign(size_t(A) * m, 0);
    for (int64_t r = 0; r < A * m; ++r) {
      const double *v = V + r * B;
      for (int64_t q = 0; q < B; ++q)
        if (v[q] != 0.0) {
          nz[r] = 1;
          break;
        }
    }
    if (B > 1) {
      parallel_rows(A * m, [&](int64_t item) {
        const int64_t alpha = item / m;
        const int i = int(item % m);
        double *w = W.data() + item * B;
        std::fill(w, w + B, 0.0);
        for (int a = 0; a < m; ++a) {
          const double c = Rs[int64_t(a) * m + i];
          if (c == 0.0 || !nz[alpha * m + a]) continue;
          const double *v = V + (alpha * m + a) * B;
          for (int64_t q = 0; q < B; ++q) w[q] += c * v[q];
        }
      });
    } else {
      parallel_rows(A, [&](int64_t alpha) {
        double *w = W.data() + alpha * m;
        std::fill(w, w + m, 0.0);
        for (int a = 0; a < m; ++a) {
          const double v = V[alpha * m + a];
          if (v == 0.0) continue;
          const double *Ra = &Rs[int64_t(a) * m];
          for (int i = 0; i < m; ++i)
            if (Ra[i] != 0.0) w[i] += Ra[i] * v;
        }
      });
    }
    std::copy(W.begin(), W.end(), V);
  }
}

// ----------------------------------------------------------- terms
// sort an operator string to index order (spin-orbital ascending, creation
// before annihilation on the same index); returns the permutation sign.
int sort_ops(int *e, int n) {
  int sign = 1;
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0; --j) {
      const int ka = e[j - 1] >> 1, kb = e[j] >> 1;
      const bool swap = (ka > kb) || (ka == kb && (e[j - 1] & 1) < (e[j] & 1));
      if (!swap) break;
      std::swap(e[j - 1], e[j]);
      sign = -sign;
    }
  return sign;
}

void Hamiltonian::build(int n_sites, int spin_half, const double *T, const double *V, const int32_t *ijkl,
                        const double *val, int64_t nnz, QN target_) {
  n = n_sites;
  ns = spin_half ? 2 : 1;
  d = 1 << ns;
  nso = ns * n;
  target = target_;
  terms.clear();
  n1 = n2 = 0;
  double tmax = 0.0;
  for (int64_t i = 0; i < int64_t(nso) * nso; ++i) tmax = std::max(tmax, std::fabs(T[i]));
  // Hermiticity of T
  for (int p = 0; p < nso; ++p)
    for (int q = 0; q < nso; ++q)
      MDMRG_REQUIRE(std::fabs(T[p * nso + q] - T[q * nso + p]) <= 1e-12 * std::max(1.0, tmax), -1,
                    "Hamiltonian: T is not symmetric");
  // dense V view (from dense or COO input)
  std::vector<double> Vd;
  const double *Vp = V;
  const int64_t N4 = int64_t(nso) * nso * nso * nso;
  if (!V) {
    Vd.assign(N4, 0.0);
    for (int64_t e = 0; e < nnz; ++e) {
      const int p = ijkl[4 * e], q = ijkl[4 * e + 1], r = ijkl[4 * e + 2], s = ijkl[4 * e + 3];
      MDMRG_REQUIRE(p >= 0 && q >= 0 && r >= 0 && s >= 0 && p < nso && q < nso && r < nso && s < nso, -1,
                    "Hamiltonian: COO index out of range");
      Vd[((int64_t(p) * nso + q) * nso + r) * nso + s] += val[e];
    }
    Vp = Vd.data();
  }
  auto v4 = [&](int p, int q, int r, int s) { return Vp[((int64_t(p) * nso + q) * nso + r) * nso + s]; };
  double vmax = 0.0;
  for (int64_t e = 0; e < N4; ++e) vmax = std::max(vmax, std::fabs(Vp[e]));
  const double vtol = 1e-12 * std::max(1.0, vmax);
  for (int p = 0; p < nso; ++p)
    for (int q = 0; q < nso; ++q)
      for (int r = 0; r < nso; ++r)
        for (int s = 0; s < nso; ++s)
          MDMRG_REQUIRE(std::fabs(v4(p, q, r, s) - v4(s, r, q, p)) <= vtol, -1,
                        "Hamiltonian: V[p,q,r,s] != V[s,r,q,p] (not Hermitian)");
  const double drop = 1e-15 * std::max(1.0, std::max(tmax, vmax));
  // one-body
  for (int p = 0; p < nso; ++p)
    for (int q = 0; q < nso; ++q) {
      const double c = T[p * nso + q];
      if (std::fabs(c) <= drop) continue;
      Term t;
      t.n = 2;
      t.e[0] = 2 * p + 1;
      t.e[1] = 2 * q;
      t.c = c * sort_ops(t.e, 2);
      terms.push_back(t);
      ++n1;
    }
  // two-body, antisymmetrised over p<q, r<s
  for (int p = 0; p < nso; ++p)
    for (int q = p + 1; q < nso; ++q)
      for (int r = 0; r < nso; ++r)
        for (int s = r + 1; s < nso; ++s) {
          const double g = v4(p, q, r, s) - v4(q, p, r, s) - v4(p, q, s, r) + v4(q, p, s, r);
          if (std::fabs(g) <= drop) continue;
          Term t;
          t.n = 4;
          t.e[0] = 2 * p + 1;
          t.e[1] = 2 * q + 1;
          t.e[2] = 2 * r;
          t.e[3] = 2 * s;
          t.c = g * sort_ops(t.e, 4);
          terms.push_back(t);
          ++n2;
        }
  // every term must conserve the quantum numbers of the symmetry
  for (const Term &t : terms) {
    QN q;
    for (int i = 0; i < t.n; ++i) q = q + q_of_op(t.e[i]);
    MDMRG_REQUIRE(q == QN(), -1,
                  spin_half ? "Hamiltonian: a term changes (N_up, N_down); U(1)xU(1) needs spin-conserving T, V"
                            : "Hamiltonian: a term changes the particle number");
  }
  // reachability of the target
  const QN maxq = spin_half ? QN(n, n) : QN(n, 0);
  MDMRG_REQUIRE(target.a >= 0 && target.b >= 0 && target.a <= maxq.a && target.b <= maxq.b, -1,
                "Hamiltonian: target sector unreachable");
}

QN Hamiltonian::q_of_op(int e) const {
  const int p = e >> 1;
  const int sgn = (e & 1) ? 1 : -1;
  if (ns == 2) return (p & 1) ? QN(0, sgn) : QN(sgn, 0);
  return QN(sgn, 0);
}

QN Hamiltonian::q_of_state(int s) const {
  if (ns == 2) return QN(s & 1, (s >> 1) & 1);
  return QN(s & 1, 0);
}

// d x d matrix (row = bra) of the ordered product e[0] e[1] ... e[k-1] of
// elementary operators of one site (local Jordan-Wigner signs)
std::vector<double> Hamiltonian::site_matrix(int site, const int *e, int k) const {
  std::vector<double> M(d * d, 0.0);
  for (int t = 0; t < d; ++t) {
    int s = t;
    double amp = 1.0;
    bool ok = true;
    for (int j = k - 1; j >= 0; --j) {
      const int p = e[j] >> 1, dag = e[j] & 1;
      const int sig = p - ns * site;
      const int occ = (s >> sig) & 1;
      if (occ == dag) {
        ok = false;
        break;
      }
      if (__builtin_popcount(s & ((1 << sig) - 1)) & 1) amp = -amp;
      s ^= (1 << sig);
    }
    if (ok) M[s * d + t] += amp;
  }
  return M;
}

}  // namespace mdmrg
