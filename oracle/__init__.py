"""Plain CPU FP64 oracle for the mode-optimized DMRG hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or execute anything under ``oracle/``;
only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use it.

The oracle is deliberately slow and literal:

* ``integrals``  -- Eq. (1)-(3) and the mode transformation of Sec. II.B,
  written out as dense FP64 arrays (lattice, momentum basis, rotation).
* ``ed``         -- exact diagonalisation in a fixed particle-number sector
  (Fock bitstrings, Jordan-Wigner signs), used to pin everything else.
* ``dmrg``       -- a two-site DMRG (Sec. II.A) whose renormalised blocks are
  kept as *explicit* Fock-space basis vectors, so that the effective
  Hamiltonian product is the plain projection  P^T H P psi.  It shares no
  code with, and uses none of the operator bookkeeping of, the GPU path.
* eigenpairs -- ``dmrg.TwoSiteProblem.lowest`` takes the lowest eigenpair of
  H_eff by its plain definition (dense ``eigh`` for small dimensions, scipy's
  Lanczos ``eigsh`` otherwise); the library's Davidson (Sec. II.A names
  Lanczos or Davidson) is compared with that eigenvalue, not with another
  Davidson.
* ``split``      -- the split-precision product models (FP32, 3xBF16
  hi/lo and 6xBF16 hi/mid/lo products) evaluated in FP64, for the kernel
  tests of those forms.
* ``su2``        -- Clebsch-Gordan coefficients and 6j symbols in exact
  rational arithmetic (Racah formulas), 9j symbols, SU(2) multiplet bases
  of small spin-1/2 fermion blocks, Wigner-Eckart reduced elements, the 6j
  product rule of coupled operators and the spin-adapted two-block
  superblock of a Hubbard model (the algebra of the spin-adapted form,
  Sec. IV).
* ``rdm``        -- one- and two-particle reduced density matrices of an
  explicit Fock-space state, the energy of Eq. (1) from them and the
  charge-density-wave order parameter (Sec. II.B, III.C).
* ``modeopt``    -- mode rotations of an explicit Fock-space state (the
  exponential of the one-body generator), the half-Renyi entropy of a
  bipartition and the two-mode micro-iteration that lowers it (Sec. II.B).
* ``ozaki``      -- FP64 products from exact integer products of 8-bit
  slices with per-row and per-column exponents (the model of an
  FP64-accurate split form on the integer matrix units; not in the paper).
* ``mutual``     -- one- and two-mode entropies, mutual information, total
  correlation and correlation distance, natural modes, the Fiedler
  ordering, the DEAS order and the HF reference taken after the last sweep
  (Sec. II.B).

Pins (closed forms, brute force on tiny inputs, basis invariance) live in
``tests/test_oracle_*.py``.
"""
