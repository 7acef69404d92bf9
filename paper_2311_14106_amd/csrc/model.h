// Model layer: lattice builders, mode rotation, canonical term list.
#pragma once
#include "internal.h"

namespace mdmrg {

int lattice_nso(int model, int Lx, int Ly);
void build_lattice(int model, int basis, int Lx, int Ly, double t, double u, double *T, double *V);
void rotate_modes(int n, int spin_half, const double *R, double *T, double *V);
int sort_ops(int *e, int n);

// One operator term c * e[0] ... e[n-1] of Eq. (1); elementary operator
// e = 2*p + dagger, list in index order (spin-orbital ascending, creation
// first on equal index); the permutation sign is folded into c.
struct Term {
  double c = 0.0;
  int n = 0;
  int e[4] = {0, 0, 0, 0};
};

struct Hamiltonian {
  int n = 0, ns = 1, d = 2, nso = 0;
  QN target;
  std::vector<Term> terms;
  int64_t n1 = 0, n2 = 0;
  void build(int n_sites, int spin_half, const double *T, const double *V, const int32_t *ijkl,
             const double *val, int64_t nnz, QN target);
  int site_of(int e) const { return (e >> 1) / ns; }
  QN q_of_op(int e) const;
  QN q_of_state(int s) const;
  std::vector<double> site_matrix(int site, const int *e, int k) const;
};

}  // namespace mdmrg
