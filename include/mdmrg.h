/*
 * mdmrg -- MI355X (gfx950) hot path of mode-optimized ab initio DMRG.
 *
 * C ABI of libmdmrg.so.  Every entry point returns an int status (0 = OK,
 * negative = error, see MDMRG_E*) and never throws across the boundary; the
 * text of the last error of a context is returned by mdmrg_last_error().
 * Host arrays passed in are copied (the caller keeps ownership).  Device
 * pointers passed in (x, y, diagonal buffers) are caller-owned allocations on
 * the context's device, laid out as reported by mdmrg_psi_layout().
 * All device work runs on the context's stream; calls that return host
 * scalars synchronise that stream.  A context is used by one host thread at a
 * time.
 *
 * Model (Eq. (1), Sec. II.A):
 *     H = sum_pq T[p,q] a+_p a_q + sum_pqrs V[p,q,r,s] a+_p a+_q a_r a_s
 * literal sums, no implied 1/2, real FP64 parameters, p a spin-orbital index.
 * Spinless fermions: one spin-orbital per site, U(1) particle number.
 * Spin-1/2 fermions: spin-orbital p = 2*site + sigma (sigma 0 = up,
 * 1 = down), local basis {0, up, down, up+down} encoded as bitmask
 * s = n_up | (n_down << 1) (Eq. (4)), U(1) x U(1) (N_up, N_down).
 *
 * Exchange format of matrix product states (Eq. (4)):
 *   bond i (0..n) sits left of site i; its sectors carry the quantum numbers
 *   of sites [0, i): (N, 0) spinless or (N_up, N_down), listed in ascending
 *   lexicographic order.  Bond 0 is {(0,0): 1}; bond n is {target: 1}.
 *   Site tensor i has one dense block per (l, s, r) with
 *   Q_r = Q_l + q(s), l a sector of bond i, r of bond i+1, of shape
 *   m_l x m_r, row-major; blocks are concatenated site by site in
 *   lexicographic (l, s, r) order.
 *   The two-site wave function at bond (l, l+1) has one block per
 *   (a, s1, s2, b), a a sector of bond l, b of bond l+2,
 *   Q_a + q(s1) + q(s2) = Q_b, shape m_a x m_b row-major, packed in
 *   lexicographic (a, s1, s2, b) order without padding.  The basis state of
 *   element (a,i; s1; s2; b,j) is |a,i>|s1>|s2>|b,j> with the creation
 *   operators of the left block leftmost (Jordan-Wigner chain order).
 */
#ifndef MDMRG_H
#define MDMRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mdmrg_ctx_s *mdmrg_ctx;

enum {
  MDMRG_OK = 0,
  MDMRG_EINVAL = -1,   /* bad argument, shape or non-Hermitian input       */
  MDMRG_ENOMEM = -2,   /* device or host allocation failed                  */
  MDMRG_EDEVICE = -3,  /* HIP / rocSOLVER error, or NaN detected on device  */
  MDMRG_ESTATE = -4,   /* call out of order (no Hamiltonian, no MPS, ...)   */
  MDMRG_ENOCONV = -5,  /* Davidson reached max_iter; best estimate returned */
  MDMRG_EUNSUP = -6    /* valid request the library does not implement      */
};

enum { MDMRG_MODEL_SPINLESS = 0, MDMRG_MODEL_HUBBARD = 1 };
enum { MDMRG_BASIS_REAL = 0, MDMRG_BASIS_MOMENTUM = 1 };
enum { MDMRG_FP64 = 0, MDMRG_FP32 = 1, MDMRG_BF16X3 = 2, MDMRG_BF16X6 = 3 };

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` (the device that runs the
 * effective-Hamiltonian products of the DMRG steps, Sec. II.A and III.B).
 * hip_stream: the caller's hipStream_t on that device (for instance the
 * stream of a torch.cuda.Stream), on which every device call of the context
 * is then queued; the caller keeps ownership and must not destroy it before
 * mdmrg_destroy.  NULL: the context creates a blocking, default-priority
 * stream of its own.  *out receives the handle; on failure *out is NULL and
 * mdmrg_last_error(NULL) says why (EINVAL for a stream of another device).
 * The context may hold up to 95% of the device memory free at this call (see
 * MDMRG_OPT_MEMORY_BUDGET); a call that would need more fails with
 * MDMRG_ENOMEM. */
int mdmrg_create(mdmrg_ctx *out, int device, void *hip_stream);
/* Release every device and host resource of the context.  NULL is a no-op. */
void mdmrg_destroy(mdmrg_ctx ctx);
/* Context-owned, NUL-terminated text of the last error ("" if none). */
const char *mdmrg_last_error(mdmrg_ctx ctx);
/* Library version string (static storage). */
const char *mdmrg_version(void);

/* ----------------------------------------------- model parameters (host) */

/* Number of spin-orbitals of a model on an Lx x Ly torus. */
int mdmrg_lattice_nso(int model, int Lx, int Ly);

/* Eq. (2) (model HUBBARD, u = U) or Eq. (3) with t' = 0 (model SPINLESS,
 * u = V) on an Lx x Ly torus (Sec. II.A).  Hopping enters as -t.
 * basis REAL: sites in row-major snake order, bonds (x,y)-(x+1,y) and
 * (x,y)-(x,y+1) with periodic wrap, each once.  basis MOMENTUM: plane-wave
 * modes k = 2 pi (a/Lx, b/Ly) ordered by eps_k = -2t(cos kx + cos ky)
 * ascending, ties by label b*Lx+a; spinless V[k1,k2,k3,k4] =
 * (u/N)(cos qx + cos qy) delta(k1+k2=k3+k4), q = k3-k2; Hubbard
 * V[(k1 up),(k2 dn),(k3 dn),(k4 up)] = (u/N) delta(k1+k2=k3+k4).
 * T (nso*nso) and V (nso^4), row-major, caller-allocated, overwritten. */
int mdmrg_build_lattice(int model, int basis, int Lx, int Ly, double t, double u,
                        double *T, double *V);

/* Mode transformation on the parameters (Sec. II.B): old modes
 * c_a = sum_i R[a,i] d_i, R real orthogonal n_modes x n_modes row-major.
 * T <- R^T T R, V[i,j,k,l] <- sum R[a,i]R[b,j]R[c,k]R[d,l] V[a,b,c,d].
 * spin_half != 0 applies R to both spin components (p = 2*mode + sigma).
 * T and V are updated in place.  EINVAL if R is not orthogonal (1e-10). */
int mdmrg_rotate_modes(int n_modes, int spin_half, const double *R, double *T, double *V);

/* ------------------------------------------------------------- Hamiltonian */

/* Set Eq. (1) on n_sites sites.  spin_half selects the local dimension
 * (2 or 4) and the symmetry (U(1) or U(1)xU(1)); T is nso x nso, V nso^4
 * dense row-major (nso = n_sites or 2*n_sites).  target = (N, 0) or
 * (N_up, N_down).  EINVAL if T != T^T or V[p,q,r,s] != V[s,r,q,p] beyond
 * 1e-12 * max|.|, or if the target is unreachable.  Invalidates the MPS. */
int mdmrg_set_hamiltonian(mdmrg_ctx ctx, int n_sites, int spin_half, const double *T,
                          const double *V, int target_a, int target_b);

/* Same with V in coordinate form: nnz entries (p,q,r,s) = ijkl[4*e..4*e+3],
 * value val[e]; repeated entries add up (the sparse interaction lists of
 * the lattice models of Eq. (2)-(3)).  Same validation as the dense form,
 * plus EINVAL for an index outside [0, nso). */
int mdmrg_set_hamiltonian_coo(mdmrg_ctx ctx, int n_sites, int spin_half, const double *T,
                              int64_t nnz, const int32_t *ijkl, const double *val,
                              int target_a, int target_b);

/* Number of operator terms of the canonical (antisymmetrised) form of the
 * Hamiltonian of Eq. (1) set last: one-body and two-body strings. */
int mdmrg_n_terms(mdmrg_ctx ctx, int64_t *n_one_body, int64_t *n_two_body);

/* ------------------------------------------------------------------- MPS */

/* Load an MPS (Eq. (4), Sec. II.B) in the exchange format above.
 * n_sect[n+1] sector counts per bond; sect_qn[2*S] and sect_dim[S] for all S sectors of all bonds in bond
 * order; data = site tensors (n_data doubles).  Sites left of the bond later
 * prepared are used as left isometries, sites right of it as right
 * isometries. */
int mdmrg_set_mps(mdmrg_ctx ctx, const int32_t *n_sect, const int32_t *sect_qn,
                  const int32_t *sect_dim, const double *data, int64_t n_data);

/* Export the MPS site tensors in the exchange format of mdmrg_set_mps
 * (the sector lists of the bonds are those of mdmrg_get_bond): *n_needed
 * receives the number of doubles; with data != NULL (n_data >= that) the
 * tensors are copied to the host buffer.  After decimation the exported
 * sites are the library's current tensors: the isometries left and right
 * of the current bond; the two-site centre itself lives in the Davidson
 * vector, not in the tensors. */
int mdmrg_get_mps(mdmrg_ctx ctx, double *data, int64_t n_data, int64_t *n_needed);

/* Sector list of bond i of the MPS (Eq. (4): the quantum-number blocks of
 * the bond index, dimensions D_i split by sector): query with
 * qn = dim = NULL to get *n_sect. */
int mdmrg_get_bond(mdmrg_ctx ctx, int bond, int32_t *n_sect, int32_t *qn, int32_t *dim);

/* ------------------------------------------------------------------- bond */

enum {
  MDMRG_OPT_KEEP_ENVS = 1,     /* which block operators mdmrg_prepare_bond keeps at bond l
                                  (large-D workloads; a block that is needed later and
                                  was dropped is rebuilt from the chain end):
                                  1 (default): every block built;
                                  0: this bond's and one step either way (left blocks at
                                  bonds l-1 and l, right blocks at l+2 and l+3);
                                  2: a walk to the right (left block at l, every right
                                  block at bonds >= l+2);
                                  3: one step to the right (left block at l, right blocks
                                  at l+2 and l+3).
                                  Right blocks are built before left ones, and the
                                  operators a renormalisation forms on the fly are made
                                  in batches of at most 2^28 doubles */
  MDMRG_OPT_SCRATCH_LIMIT = 2, /* doubles of intermediate storage per product pass
                                  (default 2^30); larger values mean fewer passes */
  MDMRG_OPT_GRAPH = 3,         /* 1: after the first products of a bond (which also
                                  tune the kernel's tile variant per launch), capture
                                  the bond's H_eff x launch sequence per precision in a
                                  HIP graph and replay it for every later product
                                  (x and y staged through context buffers for FP64);
                                  0 (default): launch eagerly */
  MDMRG_OPT_COMPRESS = 4,      /* 1 (default): the N^L x O_s x C^R products of a bond are
                                  grouped by site operator s and quantum-number shift, and
                                  each group is reduced by an interpolative decomposition
                                  of its coefficient matrix (relative rank cut 1e-14,
                                  reconstruction checked to 1e-12) to skeleton products
                                  with on-the-fly left combinations; 0: one product per
                                  left operator (takes effect at the next bond prepared) */
  MDMRG_OPT_GEMM_VARIANT = 5,  /* -1 (default): every grouped-GEMM plan times its first
                                  launches on the tile variants in turn and keeps the
                                  fastest; 0..3: every launch of the context uses that
                                  variant (k_gemm, k_gemm_w16, k_gemm_w4, k_gemm_t128;
                                  all give bitwise identical results) */
  MDMRG_OPT_MEMORY_BUDGET = 6, /* bytes of device memory the context may hold (its
                                  operator arenas, wave-function buffers, scratch and
                                  plans); an allocation beyond it fails with
                                  MDMRG_ENOMEM before reaching the allocator.  0 (and
                                  the upper limit): 95% of the device memory free at
                                  mdmrg_create */
  MDMRG_OPT_DAVIDSON_KEEP = 7, /* Ritz vectors (lowest first) kept when the Davidson
                                  subspace reaches m_max and is restarted, 2..58 (default
                                  2; at most m_max - 2 are kept) */
  MDMRG_OPT_DAVIDSON_OLSEN = 8, /* 1: Olsen's correction vector t = P r - eps P x,
                                  eps = (x.P r)/(x.P x), P = (theta - diag H_eff)^-1;
                                  0 (default): t = P r */
  MDMRG_OPT_MIXED_LADDER = 9,  /* 1: a mixed solve with prec_split MDMRG_BF16X3 runs an
                                  FP32 stage (to tol_split or its own noise floor)
                                  between the 3xBF16 and the FP64 stages; 0 (default):
                                  3xBF16 then FP64 */
  MDMRG_OPT_MIXED_HANDOVER = 10, /* 1..16: each stage of a mixed solve after the first
                                  starts from this many lowest Ritz vectors of the
                                  previous stage (one product each in its own precision);
                                  1 (default): from the eigenvector estimate alone */
  MDMRG_OPT_MIXED_CORRECT = 11  /* 1: when the split stages of a mixed solve stop with
                                  an FP64 residual above 4 tol, up to four
                                  defect-corrected split stages follow (see
                                  mdmrg_davidson_mixed) before the FP64 Davidson
                                  stage; 0 (default): FP64 Davidson directly */
};
/* Set a context option (EINVAL for unknown options or bad values).
 * With the environment variable MDMRG_VERBOSE set, the library prints
 * progress lines on stderr: each block environment built, the timing of the
 * Tables step, the residual after each Davidson product. */
int mdmrg_set_option(mdmrg_ctx ctx, int option, int64_t value);

/* Make bond (l, l+1) current: build (on the device) the renormalised
 * operators of the left block (sites < l) and the right block
 * (sites > l+1) from the MPS by repeated renormalisation (Sec. II.A), then
 * the "Tables" of the step (Sec. III.B, the overhead category of Fig. 7):
 * sector lists, the wave-function layout and the task lists of the
 * effective Hamiltonian.  EINVAL if l + 1 is not a site, ESTATE without a
 * Hamiltonian and an MPS, ENOMEM if the operators exceed the budget. */
int mdmrg_prepare_bond(mdmrg_ctx ctx, int l);

/* Layout of the current two-site vector (the wave function of the local
 * two-site optimisation step, Sec. II.A).  *n_elem = total doubles,
 * *n_blk = number of blocks; if desc != NULL it receives 8 int32 per block:
 * (a, s1, s2, b, m_a, m_b, offset_lo, offset_hi). */
int mdmrg_psi_layout(mdmrg_ctx ctx, int64_t *n_elem, int32_t *n_blk, int32_t *desc);

/* y = H_eff x at the current bond: the product of the effective
 * Hamiltonian, built from the renormalised block operators of the left and
 * right blocks and the two site operators with the integrals of Eq. (1),
 * with a two-site vector (Sec. II.A; the Diag_H work of Sec. III.B, Fig. 8).
 * x, y: caller-owned device buffers of n_elem doubles on the context's
 * device, layout of mdmrg_psi_layout, must not alias (EINVAL); the library
 * cannot check their length, so a shorter buffer is read or written past its
 * end.  ESTATE without a current bond.  prec MDMRG_FP64 is the plain form;
 * MDMRG_FP32 (split form) runs every GEMM on FP32 shadows of the operators
 * and of x with FP32 MFMA accumulation, y returned in FP64; MDMRG_BF16X3
 * (split form) reads the same FP32 shadows and forms every product from
 * BF16 parts, hi = RNE(v), lo = RNE(v - hi) of each operand element v, as
 * hi*lo + lo*hi + hi*hi with FP32 accumulation (about 16 significant bits
 * per operand, BF16 MFMA rate), y returned in FP64; MDMRG_BF16X6 (split
 * form) splits every element into three BF16 parts, hi = RNE(v),
 * mid = RNE(v - hi), lo = RNE(v - hi - mid), and sums the six products
 * hi*lo + lo*hi + mid*mid + hi*mid + mid*hi + hi*hi in FP32 (about the
 * accuracy of FP32 operands at the BF16 MFMA rate).  Other values: EUNSUP. */
int mdmrg_heff_apply(mdmrg_ctx ctx, int prec, const double *x, double *y);

/* Diagonal of H_eff at the current bond (Sec. II.A; the preconditioner of
 * the Davidson iteration) into the caller-owned device buffer d of n_elem
 * doubles.  ESTATE without a current bond. */
int mdmrg_heff_diag(mdmrg_ctx ctx, double *d);

/* Cost of one H_eff x at the current bond (the complexity measure of
 * Sec. III.A, counted in FLOP): algorithmic FLOP (sum over GEMM
 * tasks of 2mnk in the chosen order, no padding, identity products not
 * counted), algorithmic bytes (each distinct operand block read once, each
 * output block written once, intermediates written and read once), the
 * number of operator products (terms) and of GEMM segments.  Any output
 * pointer may be NULL. */
int mdmrg_heff_cost(mdmrg_ctx ctx, double *flop, double *bytes, int64_t *n_terms, int64_t *n_gemm);

/* Shape profile of one H_eff x at the current bond (Sec. III.B: the block
 * sizes that decide the GPU efficiency; the workload shape the
 * grouped kernels see): algorithmic FLOP of its GEMMs binned by the smaller
 * output side min(m, n), bins [1,16) [16,32) [32,48) [48,64) [64,128)
 * [128,256) [256,512) [512,inf); flop_by_bin must hold 8 doubles.  Sums to
 * the FLOP of mdmrg_heff_cost.  ESTATE before mdmrg_prepare_bond. */
int mdmrg_heff_histogram(mdmrg_ctx ctx, double *flop_by_bin);

/* Davidson for the lowest eigenpair of H_eff (the iterative
 * diagonalisation of the effective Hamiltonian in each local step,
 * Sec. II.A; its convergence threshold is the epsilon of Sec. III.A-B),
 * FP64 on device.  x (device, n_elem) holds the start vector on entry
 * (normalised inside; if zero, a seeded random vector is used) and the
 * eigenvector on exit.  Stops at ||H x - theta x||_2 <= tol with
 * ||x|| = 1.  Returns ENOCONV, with the best estimate in *energy / x, after
 * max_iter matrix-vector products or when the subspace admits no new
 * direction before tol is reached.  EDEVICE if the start vector or the
 * residual is not finite (NaN / Inf in x or in the operators).
 * m_max in [3, 60]: subspace size before a thick restart to 2 vectors. */
int mdmrg_davidson(mdmrg_ctx ctx, double *x, double tol, int max_iter, int m_max,
                   double *energy, double *resid, int *n_matvec);

/* Mixed-precision Davidson (the products beyond the FP64 ceiling of Sec. IV
 * and Fig. 2, with the final eigenpair held to FP64 accuracy): a Davidson
 * solve whose products use the split form prec_split (MDMRG_FP32,
 * MDMRG_BF16X3 or MDMRG_BF16X6) until its residual reaches tol_split or
 * stops decreasing (no 10% gain over 4 products once within 2f, over 24
 * within 20f, over 64 elsewhere), then (MDMRG_OPT_MIXED_LADDER, 3xBF16
 * only) an FP32 stage the same way.  f is the noise floor of the split
 * operator, measured with one split and one FP64 product of the normalised
 * start vector v: f = |(H_split - H) v| / |H v| * |v.H v|.
 * Then (MDMRG_OPT_MIXED_CORRECT; off by default) up to four defect-corrected
 * rounds: one FP64 product of the current vector x0 gives its FP64
 * residual -- if <= tol the solve ends there, with the FP64 Rayleigh
 * quotient x0.H x0 as the energy -- and, with one split product, the defect
 * d = H x0 - H_split x0; a split Davidson on H_split + d x0^T + x0 d^T -
 * (x0.d) x0 x0^T (which reproduces H x0 exactly) then runs to tol / 2 or
 * until 8 products bring no 10% gain.
 * Once the FP64 residual is within 4 tol (or after four rounds), an FP64
 * Davidson from that vector, reusing its FP64 product, until the FP64
 * residual <= tol (without the option: directly after the split stages).
 * *n_mv64 and *n_mv_split count the products of each kind (the floor probe
 * included). */
int mdmrg_davidson_mixed(mdmrg_ctx ctx, double *x, double tol, int prec_split, double tol_split,
                         int max_iter, int m_max, double *energy, double *resid, int *n_mv64,
                         int *n_mv_split);

/* Reduced-density-matrix truncation of the two-site vector x (the Diag_D
 * category of Sec. III.B; the bond dimension D of Sec. II.A):
 * direction +1 replaces site l by a left isometry and bond l+1 by the kept
 * states of the left enlarged block; -1 replaces site l+1 by a right
 * isometry.  rho is the density matrix of the normalised state
 * x / |x| (trace 1), so any nonzero scale of x gives the same result; EINVAL
 * for a zero x, EDEVICE for a non-finite one.  Keeps min(D, available) states
 * ranked by eigenvalue.  Outputs truncation error (discarded weight), von
 * Neumann entropy -Tr rho ln rho and half-Renyi entropy 2 ln Tr sqrt(rho)
 * (Sec. II.B), any may be NULL. */
int mdmrg_decimate(mdmrg_ctx ctx, const double *x, int D, int direction, double *trunc_err,
                   double *s_vn, double *s_half);

/* Renormalisation (the renormalised block operators of Sec. II.A; Ren_l /
 * Ren_r of Sec. III.B): after mdmrg_decimate(direction) at bond
 * (l, l+1), build on the device every operator of the grown block (left
 * block of sites <= l for +1, right block of sites >= l+1 for -1) from the
 * new isometry, then make bond (l+direction, l+direction+1) current
 * (as mdmrg_prepare_bond).  prec selects the arithmetic of the
 * renormalisation GEMMs: MDMRG_FP64 (plain); MDMRG_FP32, MDMRG_BF16X3 or
 * MDMRG_BF16X6 (split forms, as in mdmrg_heff_apply, on FP32 copies of the
 * source operators and the isometry, FP32 accumulation).  The new operators are
 * stored as FP64 either way; a split form perturbs them at its rounding
 * level (about 1e-7 relative for FP32, 1e-5 for 3xBF16), a first-order
 * change of H_eff that later FP64 products do not remove.  Other prec:
 * EUNSUP.  ESTATE if the last call at this bond was not mdmrg_decimate with
 * the same direction. */
int mdmrg_renormalize(mdmrg_ctx ctx, int direction, int prec);

/* Start vector of the new current bond (the StVec category of Sec. III.B):
 * x_new (n_elem of the new
 * layout) = the two-site vector x_old of the previous bond (its layout)
 * written in the new basis,  psi' = P'^T P psi.  Valid right after
 * mdmrg_renormalize; x_old and x_new are caller-owned device buffers. */
int mdmrg_stvec(mdmrg_ctx ctx, const double *x_old, double *x_new);

/* Finite two-site DMRG sweeps (Sec. II.A) from the current MPS (a right
 * then a left half-sweep per sweep), bond dimension
 * D_schedule[min(k, n_sched-1)] in sweep k, Davidson tolerance tol, FP64
 * throughout.  energies receives the final energy of each sweep (n_sweeps
 * doubles, may be NULL).  Returns ENOCONV after completing the sweeps if a
 * Davidson solve missed tol (mdmrg_last_error gives the count). */
int mdmrg_sweep(mdmrg_ctx ctx, int n_sweeps, const int *D_schedule, int n_sched, double tol,
                double *energies);

/* The grouped sector-block GEMM that carries every dense contraction of the
 * path (H_eff products, renormalisation, density matrices: the block
 * operations distributed over GPUs in Sec. III.B, Fig. 7), exposed for
 * direct use.  For each output o (8 int64 per output:
 * slot, offset, m, n, ldc, seg_begin, seg_count, accumulate):
 *   C_o = (accumulate ? C_o : 0) + sum_{s in segments of o} alpha[s] op(A_s) op(B_s)
 * with segment s given by 8 int64: a_slot, a_offset, lda, b_slot, b_offset,
 * ldb, k, flags (1 = A transposed, 2 = B transposed, 4 = A is the identity).
 * All matrices are FP64 row-major inside caller-owned device buffers
 * bases[0..n_bases-1] (n_bases <= 8) of base_len[i] doubles; offsets are in
 * elements; m, n < 2^30.  Every access range is checked on the host first
 * (EINVAL); an operand whose rows x leading dimension within one 32-deep K
 * step reaches 2^31 elements is refused (EUNSUP).
 * Outputs must not overlap each other or any operand of the call. */
int mdmrg_gemm_grouped(mdmrg_ctx ctx, int n_bases, const double *const *bases, const int64_t *base_len,
                       int64_t n_out, const int64_t *out_desc, int64_t n_seg, const int64_t *seg_desc,
                       const double *alpha);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * grouped GEMM of mdmrg_gemm_grouped, same descriptors, range checks and
 * results, without any device allocation.  The segment, output and tile
 * descriptors are staged in a static per-GPU array of
 * MDMRG_NOALLOC_STAGING_BYTES (16 MiB) that the library holds on each GPU it
 * runs on until the process ends; a call whose descriptors and tile list
 * need more returns MDMRG_EINVAL ("above the static staging limit").  The
 * launch uses the tile variant forced by MDMRG_OPT_GEMM_VARIANT, else
 * k_gemm_w4 (no autotuning; every variant gives the same bits), and the call
 * returns after the launch has completed on the context stream.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * host threads, or contexts on other streams) race and must be serialised
 * by the caller. */
#define MDMRG_NOALLOC_STAGING_BYTES (16u << 20)
int mdmrg_gemm_grouped_noalloc(mdmrg_ctx ctx, int n_bases, const double *const *bases, const int64_t *base_len,
                               int64_t n_out, const int64_t *out_desc, int64_t n_seg, const int64_t *seg_desc,
                               const double *alpha);

/* The same grouped GEMM in a split-precision form (the arithmetic of the
 * split H_eff products: the products beyond the FP64 ceiling of Sec. IV and
 * Fig. 2, in FP32, 3xBF16 or 6xBF16): every
 * buffer holds FP32 elements (base_len[i] floats, offsets in floats), alpha
 * is rounded to FP32 and folded into op(A) before the product, results are
 * FP32.  prec MDMRG_FP32: FP32 MFMA products and accumulation.  prec
 * MDMRG_BF16X3: each element v of alpha op(A) and of op(B) is split into
 * hi = RNE_bf16(v), lo = RNE_bf16(v - hi) and the product is accumulated
 * in FP32 as hi*lo + lo*hi + hi*hi.  prec MDMRG_BF16X6: three parts,
 * mid = RNE_bf16(v - hi), lo = RNE_bf16(v - hi - mid), and the six products
 * hi*lo + lo*hi + mid*mid + hi*mid + mid*hi + hi*hi.  Other prec: EUNSUP;
 * descriptors and
 * range checks as for mdmrg_gemm_grouped (EINVAL). */
int mdmrg_gemm_grouped_split(mdmrg_ctx ctx, int prec, int n_bases, const float *const *bases,
                             const int64_t *base_len, int64_t n_out, const int64_t *out_desc, int64_t n_seg,
                             const int64_t *seg_desc, const double *alpha);

/* Wall seconds per step category (Diag_H, Ren, Tables, Diag_D, StVec,
 * Other: the categories of Sec. III.B, Fig. 7) accumulated since creation, the algorithmic FLOP of all H_eff
 * products, and HIP-event timings of the grouped-GEMM kernel launches on the
 * context stream; out must hold MDMRG_N_STATS (86) doubles:
 * [diag_h, ren, tables, diag_d, stvec, other, heff_flop, n_matvec,
 *  heff_gemm_ms, heff_gemm_launches, heff_gemm_flop,
 *  ren_gemm_ms, ren_gemm_launches, ren_gemm_flop,
 *  heff_flop_split, n_matvec_split,
 *  split_gemm_ms, split_gemm_launches, split_gemm_flop,
 *  heff_phase1_ms, heff_phase1_launches, heff_phase1_flop,
 *  grouped_ms, grouped_launches, grouped_flop (mdmrg_gemm_grouped calls),
 *  heff_kernel_ms, heff_kernel_launches, heff_kernel_flop,
 *  all_kernel_ms, all_kernel_launches,
 *  proc[prec][variant][ms, launches, flop] for prec FP64, FP32, BF16X3,
 *  BF16X6 and the tile variants k_gemm, k_gemm_w16, k_gemm_w4, k_gemm_t128
 *  (48 values), graph64_ms, graph64_launches, graph32_ms, graph32_launches,
 *  graphbf3_ms, graphbf3_launches, graphbf6_ms, graphbf6_launches]. */
#define MDMRG_N_STATS 86
/*
 * heff_gemm_* covers the accumulation (second) phase of the eager FP64
 * H_eff products, heff_phase1_* their intermediate (first) phase and
 * heff_kernel_* both; split_gemm_* the eager split-form products (FP32,
 * 3xBF16 and 6xBF16 together); all_kernel_* every kernel launch of the context (all
 * forms); proc[..] every launch of one kernel in the whole process, over
 * all contexts including destroyed ones; graph*_ are whole H_eff products
 * replayed from a captured graph (MDMRG_OPT_GRAPH). */
int mdmrg_get_stats(mdmrg_ctx ctx, double *out);

/* ------------------------------------------- mode analysis (host only) */
/*
 * The quantities computed at the end of the last sweep to set up the next
 * mode-transformation macro-iteration (Sec. II.B): one- and two-mode
 * entropies, mutual information, total correlation, correlation distance,
 * the one-particle density matrix, occupations and natural modes, the
 * Fiedler ordering, the DEAS order and the HF reference.  They run on the
 * host from plain arrays (no context, no GPU); a failure returns
 * MDMRG_EINVAL (MDMRG_ENOMEM for host memory) with the message in
 * mdmrg_last_error(NULL).  A mode is a site: one spin-orbital (spinless) or
 * the pair 2i, 2i+1 (spin_half); d = 2 or 4 local states, bit t of a local
 * state = spin-orbital t of the site occupied.
 */

/* Reduced density operators of single modes and of mode pairs of the MPS
 * given in the exchange format (site tensors of mdmrg_get_mps, sector lists
 * of mdmrg_get_bond; the state need not be normalised).  With centre >= 0
 * the state is the one whose sites centre and centre+1 are the two-site
 * wave function psi (n_psi doubles on the host, n_blk blocks described as
 * by mdmrg_psi_layout over the sectors of bonds centre and centre+2): the
 * form of the library's own state during and after a sweep, whose centre
 * lives in the Davidson vector; the exchange data of those two sites is
 * then ignored.  From the state:
 *   s_one[n]       s_i = -Tr rho_i ln rho_i;
 *   s_two[n*n]     s_ij of the pair (symmetric; s_two[i*n+i] = s_i);
 * and, each optional (NULL to skip):
 *   rho_one[n*d*d] rho_i, local state index;
 *   rho_two[n*n*d^4] rho_ij for i != j in the representation with the
 *                  spin-orbitals of i moved to the front, then those of j
 *                  (the Jordan-Wigner sign of that reordering included),
 *                  local index c_i + d*c_j; the diagonal blocks are not
 *                  written;
 *   gamma[nso*nso] gamma_pq = <a+_p a_q> over spin-orbitals p = ns*i + t;
 *   occ[nso]       <n_p>;
 *   nn[n*n]        <n_i n_j>, n_i the particle number of mode i (both
 *                  spins), the density correlations of the CDW order
 *                  parameter (Sec. III.C).
 * The contraction costs about n^2 d^2 / 2 block-sparse transfers of a
 * bond operator over one site and runs on OMP_NUM_THREADS host threads
 * (default: the hardware threads; at most 64), as does the angle search of
 * mdmrg_two_mode_rotation.  EINVAL for a layout that does not add up to
 * n_data, sectors out of order, centre blocks that do not match the sectors
 * of their bonds or break the quantum-number rule, or a zero state. */
int mdmrg_mode_analysis(int n_sites, int spin_half, const int32_t *n_sect, const int32_t *sect_qn,
                        const int32_t *sect_dim, const double *data, int64_t n_data, double *s_one,
                        double *s_two, double *rho_one, double *rho_two, double *gamma, double *occ,
                        double *nn, int centre, int n_blk, const int32_t *desc, const double *psi,
                        int64_t n_psi);

/* Charge-density-wave order parameter (Sec. III.C) in the current modes:
 * C_CDW = <(sum_i s_i n_i)^2> / N^2 = sum_ij s_i s_j nn[i*n+j] / sum_ij nn,
 * with the mode signs sign[n] (+1 on one sublattice, -1 on the other, for a
 * real-space ordering) and nn from mdmrg_mode_analysis (sum_ij <n_i n_j> =
 * N^2 in a fixed-N state).  EINVAL if nn sums to zero. */
int mdmrg_cdw_order(int n, const double *nn, const double *sign, double *c_cdw);

/* Mutual information I_ij = s_i + s_j - s_ij (I_ii = 0) into I[n*n],
 * *i_tot = sum_i s_i and *i_dist = sum_{i,j} I_ij (pos(i) - pos(j))^2 over
 * the positions pos(order[k]) = k of the modes along the chain (order NULL:
 * index order).  i_tot, i_dist may be NULL.  EINVAL if order is not a
 * permutation. */
int mdmrg_mutual_information(int n, const double *s_one, const double *s_two, const int32_t *order,
                             double *I, double *i_tot, double *i_dist);

/* Mode ordering from the Fiedler vector (the eigenvector of the second-
 * smallest eigenvalue of the Laplacian diag(sum_j I_ij) - I of the graph
 * weighted by the symmetrised I[n*n]): order[n] lists the modes by
 * ascending entry.  The vector's sign is the one that correlates non-
 * negatively with the current positions; ties keep index order.  EINVAL if
 * the graph is disconnected (the second eigenvalue vanishes) or I holds a
 * non-finite value. */
int mdmrg_fiedler_order(int n, const double *I, int32_t *order);

/* Complete-active-space vector of the DEAS warm-up: order[n] = the modes by
 * decreasing one-mode entropy s_one, ties in index order. */
int mdmrg_deas_order(int n, const double *s_one, int32_t *order);

/* HF reference configuration from the spin-orbital occupations occ[nso]:
 * config[nso] (0/1) fills the target_a most occupied spin-orbitals
 * (spin_half: the target_a most occupied up and target_b most occupied
 * down ones), ties to the lower index.  EINVAL for a target outside
 * [0, n_sites]. */
int mdmrg_hf_reference(int n_sites, int spin_half, const double *occ, int target_a, int target_b,
                       int8_t *config);

/* Natural occupation numbers occupation[nso] (descending) and natural modes
 * (the columns of modes[nso*nso], row-major; NULL to skip) of the
 * symmetrised one-particle density matrix gamma[nso*nso]. */
int mdmrg_natural_orbitals(int nso, const double *gamma, double *occupation, double *modes);

/* The two-mode micro-iteration of the mode optimisation (Sec. II.B) at a
 * bond: the two modes of the bond (the sites of s1 and s2, first and
 * second) are rotated by the angle theta, i.e. the new modes d are related
 * to the old ones by c_1 = cos(theta) d_1 - sin(theta) d_2,
 * c_2 = sin(theta) d_1 + cos(theta) d_2 (both spin components alike; on
 * Fock space U = exp(theta sum_sigma (a+_1s a_2s - a+_2s a_1s))), which is
 * the Givens matrix R of mdmrg_rotate_modes for these two modes, and the
 * half-Renyi entropy S_1/2 = 2 ln Tr sqrt(rho) of the bipartition
 * (a, s1 | s2, b) of the rotated two-site wave function is evaluated (rho
 * normalised to trace 1; its eigenvalues are the squared singular values of
 * the bipartition matrix, computed per sector by one-sided Jacobi so that
 * small ones keep their accuracy).  The blocks of psi are given as by mdmrg_psi_layout (8 int32
 * per block: a, s1, s2, b, m_a, m_b, offset_lo, offset_hi; every
 * (a, s1, s2, b) of the sector rule present, so that the rotation maps the
 * layout onto itself), psi on the host (n_elem doubles; the left and right
 * blocks are taken as orthonormal, as in the canonical form around the
 * bond).
 *   n_theta > 0: S_1/2 at theta[k] into s_half[k], and the best angle is
 *                searched on that grid;  n_theta = 0: on 64 angles
 *                covering [-pi/2, pi/2);
 * then refined by golden-section search within one grid step of the best
 * grid point: *theta_best, *s_best.  psi_rotated (NULL to skip, n_elem
 * doubles, not aliasing psi) receives the wave function rotated by
 * theta_best.  EINVAL for a descriptor outside n_elem, repeated blocks, a
 * layout that the rotation leaves, or a zero psi. */
int mdmrg_two_mode_rotation(int spin_half, int n_blk, const int32_t *desc, const double *psi, int64_t n_elem,
                            int n_theta, const double *theta, double *s_half, double *theta_best,
                            double *s_best, double *psi_rotated);

/* A sweep of two-mode micro-iterations through the chain (Sec. II.B: the
 * mode transformation built from two-mode rotations while sweeping through
 * the network).  The state is given as by mdmrg_mode_analysis with its
 * two-site centre at bond 0 (desc/psi as there; sites 2..n-1 of the
 * exchange data right isometries, sites 0 and 1 ignored).  For k = 0 .. n-2
 * the modes k, k+1 are rotated by the angle that minimises S_1/2 at bond k
 * (as mdmrg_two_mode_rotation, on the grid theta_grid[n_theta] or, with
 * n_theta = 0, on 64 angles over [-pi/2, pi/2)), then the centre moves to
 * bond k+1 by an exact factorisation (no truncation).  Outputs:
 * theta[n-1] the angles, s_half[n-1] S_1/2 of bond k after its rotation,
 * R[n*n] = G_0 G_1 ... G_{n-2} (row-major) with G_k the Givens matrix of
 * mdmrg_two_mode_rotation for modes k, k+1: mdmrg_rotate_modes(R) gives
 * the integrals in the new modes.  EINVAL as for mdmrg_mode_analysis. */
int mdmrg_rotation_sweep(int n_sites, int spin_half, const int32_t *n_sect, const int32_t *sect_qn,
                         const int32_t *sect_dim, const double *data, int64_t n_data, int n_blk,
                         const int32_t *desc, const double *psi, int64_t n_psi, int n_theta,
                         const double *theta_grid, double *theta, double *s_half, double *R);

#ifdef __cplusplus
}
#endif
#endif /* MDMRG_H */
