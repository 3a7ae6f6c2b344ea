/*
 * krylov_kernel.h -- C ABI of the MI355X (gfx950) spin-charge Krylov kernel library.
 *
 * Method: Zhang, Cawkwell, Negre, Perriot, Niklasson, "Spin-Polarized Extended
 * Lagrangian Born-Oppenheimer Molecular Dynamics" (arXiv:2303.03529).
 *   - Sec. II.G: rank-m preconditioned Krylov approximation of the kernel
 *     K = J^-1 of the residual f(n) = q[n] - n in the spin-doubled 2N space,
 *     using directional derivatives f_v = dq[n + lambda v]/dlambda - v.
 *   - Sec. II.C: Fermi-Dirac density matrix in the orthogonalized basis
 *     (H-perp = Z^T H Z, Z^T S Z = I) with one chemical potential for N_e.
 *   - Sec. III.A: spin-polarized SCC-DFTB shadow energy; its derivative gives
 *     the first-order Hamiltonians H1^sigma = 1/2 (U~ S + S U~) with per-atom
 *     potentials u^sigma = gamma v_q +/- W v_m, and Mulliken charges/moments.
 *
 * Conventions for every entry point:
 *   - Matrices and vectors are FP64, row-major, contiguous, in DEVICE memory
 *     owned by the caller (e.g. allocated through PyTorch). The library never
 *     frees or retains caller pointers past the call; kk_prepare copies or
 *     derives everything it needs into handle-owned device memory.
 *   - Vectors of length 2N are ordered (q_1..q_N, m_1..m_N): charge, then
 *     magnetization (q = n_up + n_dn, m = n_up - n_dn).
 *   - Work is enqueued asynchronously on the handle's HIP stream; outputs are
 *     valid once that stream has reached the call. Only calls that return
 *     host values (kk_get_mu, a non-NULL info, kk_profile_read) synchronize.
 *   - Errors never cross the ABI as exceptions: each call returns a kk_status
 *     and kk_last_error() gives a message (thread-local). On error nothing is
 *     enqueued unless stated otherwise.
 *   - A handle is not thread-safe; use one handle per stream.
 */
#ifndef KRYLOV_KERNEL_H
#define KRYLOV_KERNEL_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kk_handle_s *kk_handle;

typedef enum {
  KK_OK = 0,
  KK_BREAKDOWN = 1,      /* warning: the Krylov space closed early, rank_used < m */
  KK_EINVAL = -1,        /* bad argument (NULL pointer, size, offsets, m)          */
  KK_ENOMEM = -2,        /* device allocation failed                               */
  KK_EHIP = -3,          /* a HIP runtime call failed                              */
  KK_ENOTPREPARED = -4,  /* kk_prepare has not succeeded on this handle            */
  KK_ESINGULAR = -5      /* the m x m Gram matrix O is not positive definite       */
} kk_status;

/*
 * Arithmetic of the two dense transforms of each response.
 *   KK_FP64       everything in FP64 (FP64 MFMA).
 *   KK_MIXED_F16  the two transforms as three FP16 MFMA products of hi/lo
 *                 splits (~22 significant bits per operand, FP32 accumulation);
 *                 the Fermi divided differences, the chemical-potential shift,
 *                 the Mulliken sums and the Krylov m x m solve stay FP64.
 *                 Responses and kernel results agree with FP64 to ~1e-7
 *                 relative on the bcc-Fe workloads (not a guaranteed bound).
 *   KK_MIXED_BF16 the two transforms in BF16 MFMA products with FP32
 *                 accumulation and a refinement: every split operand is kept
 *                 as three BF16 pieces (hi, lo, residual; ~24 significant
 *                 bits). The hi/lo products hi*hi + hi*lo + lo*hi + lo*lo
 *                 carry ~16 bits; the refinement products over the residual
 *                 pieces, hi*res + res*hi, add the rest. All six accumulate in
 *                 one pass over the three pieces (FP32, in two levels), before
 *                 the forward's Fermi Hadamard step and the back-transform's
 *                 Mulliken sums. Six products per transform instead of
 *                 KK_MIXED_F16's three; BF16's exponent range needs no scaling.
 *                 FP64 elsewhere as above; agreement with FP64 ~1e-7 relative.
 *                 Single-system handles only (not in kk_batch_prepare).
 */
typedef enum { KK_FP64 = 0, KK_MIXED_F16 = 1, KK_MIXED_BF16 = 2 } kk_precision;

typedef struct {
  int rank_used;       /* number of Krylov directions actually used (<= m)          */
  int status;          /* KK_OK, KK_BREAKDOWN or KK_ESINGULAR                        */
  double min_pivot;    /* smallest Cholesky pivot of O (squared diagonal of L)       */
  double max_pivot;    /* largest Cholesky pivot of O                                */
  double ls_residual;  /* ||F~ c - f~|| / ||f~||: residual of the projected problem  */
} kk_info;

/* Create a handle bound to hip_stream (a hipStream_t; NULL = the null stream).
 * Allocates only host state. */
kk_status kk_create(kk_handle *h, void *hip_stream);

/* Release the handle and every device buffer it owns (synchronizes its stream). */
kk_status kk_destroy(kk_handle h);

/*
 * kk_prepare -- expansion-point setup, once per MD step (Sec. II.C).
 *   n_atoms        1 <= N <= 4096
 *   atom_offsets   HOST array of N+1 ints: orbitals of atom I are
 *                  [atom_offsets[I], atom_offsets[I+1]); offsets[0] = 0,
 *                  strictly increasing, offsets[N] = n_basis.
 *   n_basis        1 <= Nb <= 65536 (KK_EINVAL outside these ranges)
 *   S              Nb x Nb overlap matrix (symmetric positive definite)
 *   Z              Nb x Nb congruence factor with Z^T S Z = I
 *   Q_up, Q_dn     Nb x Nb orthonormal eigenvectors (columns) of Z^T H^sigma Z
 *   eps_up, eps_dn Nb eigenvalues matching the columns of Q
 *   gamma          N x N screened Coulomb matrix (symmetric)
 *   W              Stoner constant (same energy unit as eps)
 *   kT             electronic temperature (> 0, energy unit of eps)
 *   n_electrons    total electron count over both spins, 0 < N_e < 2 Nb
 *   precision      KK_FP64, KK_MIXED_F16 or KK_MIXED_BF16 (see kk_precision)
 * The library forms C^sigma = Z Q^sigma, G^sigma = S C^sigma, the occupations
 * f^sigma and solves the common chemical potential mu on the device. The
 * call allocates device memory and synchronizes the stream before returning,
 * so the inputs may be freed afterwards. Re-preparing replaces the old state.
 */
kk_status kk_prepare(kk_handle h, int n_atoms, const int *atom_offsets, int n_basis,
                     const double *S, const double *Z, const double *Q_up, const double *Q_dn,
                     const double *eps_up, const double *eps_dn, const double *gamma,
                     double W, double kT, double n_electrons, int precision);

/* Chemical potential found by kk_prepare (synchronizes the stream). */
kk_status kk_get_mu(kk_handle h, double *mu);

/*
 * density_response_batch -- first-order spin-charge response (Sec. II.G,
 * directional derivative; Sec. II.C; Sec. III.A).
 *   batch >= 1 directions v (batch x 2N, row per direction).
 *   Writes q1 (batch x 2N): q1(v) = d q[n + lambda v]/d lambda at lambda = 0,
 *   as (dq, dm). It does not subtract v; J v = q1(v) - v.
 * q1 must not overlap v.
 */
kk_status density_response_batch(kk_handle h, int batch, const double *v, double *q1);

/*
 * mulliken_project -- Mulliken projection of spin density-matrix changes
 * (Sec. III.A): dn^sigma_I = sum_{i in I} sum_j dD^sigma_ij S_ji.
 *   dD_up, dD_dn  batch x Nb x Nb each (symmetric or not)
 *   dqm           batch x 2N output (dn_up + dn_dn, dn_up - dn_dn)
 * Uses the S and atom offsets given to kk_prepare.
 */
kk_status mulliken_project(kk_handle h, int batch, const double *dD_up, const double *dD_dn,
                           double *dqm);

/*
 * krylov_kernel_apply -- rank-m preconditioned Krylov kernel (Sec. II.G):
 *   Kdelta ~ (K0 J)^-1 K0 delta = sum_{k,l<=m} v_k M_kl f~_{v_l}^T K0 delta,
 *   M = O^-1, O_kl = f~_{v_k}^T f~_{v_l}, v_k an orthonormal (modified
 *   Gram-Schmidt, two passes) basis of span{f~, (K0 J) f~, ...}, f~ = K0 delta.
 *   delta   2N residual f = q[n] - n
 *   m       1 <= m <= min(2N, 64)
 *   K0      2N x 2N preconditioner, or NULL for K0 = -I
 *   Kdelta  2N output (the caller applies -omega^2); must not overlap delta
 *   info    HOST pointer or NULL; if non-NULL the call synchronizes and fills it.
 * A direction whose orthogonalized norm drops to <= 1e-13 of its starting norm
 * ends the expansion; the result then uses rank_used < m directions and the
 * call returns KK_BREAKDOWN when info is given. delta = 0 gives Kdelta = 0.
 * If O is not positive definite, Kdelta is set to zero and info->status (and
 * the return value when info is given) is KK_ESINGULAR.
 * Unless kernel timing is on (kk_profile_enable), the update runs as one graph
 * launch on the handle's stream; the graph is captured on first use and again
 * when K0 (the pointer), m, the tolerance, the handle's buffers or the prepared
 * W or kT change (a re-prepare of the same shape, W and kT replays the existing
 * graph on the new data). The graph reads delta and writes Kdelta where they
 * are; a call whose delta or Kdelta pointer differs from the previous call's
 * first synchronizes the handle's stream and then points the graph at them.
 */
kk_status krylov_kernel_apply(kk_handle h, const double *delta, int m, const double *K0,
                              double *Kdelta, kk_info *info);

/*
 * krylov_kernel_apply_noalloc -- krylov_kernel_apply for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments, result and errors as
 * krylov_kernel_apply on a prepared handle, but the call itself allocates
 * nothing (no hipMalloc or hipFree, no library routine that allocates, no graph
 * of its own): the one-direction response workspace comes from a fixed 96 MiB
 * device array of the library, which every GPU holds until the process ends,
 * and the launches go straight onto the handle's stream. A handle whose
 * workspace does not fit is refused with KK_EINVAL before anything is enqueued
 * (handles of Nb <= 1664, e.g. 128-atom bcc Fe at Nb = 1152, fit in every
 * precision; FP64 up to Nb = 2432, KK_MIXED_F16 up to 1920). kk_prepare still
 * allocates the handle's prepared state.
 * All calls on one GPU share that array and it keeps the last call's contents:
 * calls that overlap on one GPU (two streams, or two threads) race, so the
 * caller orders them. Kernel timing (kk_profile_enable) records as usual.
 */
kk_status krylov_kernel_apply_noalloc(kk_handle h, const double *delta, int m, const double *K0,
                                      double *Kdelta, kk_info *info);

/*
 * krylov_kernel_apply_adaptive -- the same kernel with the rank chosen on the
 * device: directions are added one at a time (at most m_max) and the expansion
 * stops as soon as the projected residual ||F~ c - f~|| / ||f~|| is <= tol, the
 * residual the rank-k kernel leaves in the preconditioned Newton step. This is
 * the adaptive low-rank update used for SCF acceleration (Sec. III.C; the paper
 * uses 2-3 ranks per step and defers the criterion to earlier work, so this
 * criterion is this library's). tol = 0 behaves like krylov_kernel_apply.
 * Arguments and errors as krylov_kernel_apply; info->rank_used reports the rank.
 */
kk_status krylov_kernel_apply_adaptive(kk_handle h, const double *delta, int m_max, double tol,
                                       const double *K0, double *Kdelta, kk_info *info);

/*
 * kk_ground_state_charges -- the ground-state map q[n] at the prepared
 * expansion point (Sec. II.C, III.A): Mulliken populations of
 * D^sigma = C^sigma f^sigma C^sigma^T, written as (q, m) = (n_up + n_dn - ref,
 * n_up - n_dn) to qm (device, 2N). reference (device, N, or NULL for none) is
 * the neutral-atom electron count of each atom, the Mulliken contribution of
 * D0, so the charges come out as net charges.
 */
kk_status kk_ground_state_charges(kk_handle h, const double *reference, double *qm);

/*
 * kk_xlbomd_update -- extended-Lagrangian integration step for the electronic
 * coordinates (Sec. II.F, modified Verlet with weak dissipation):
 *   n(t+dt) = 2 n(t) - n(t-dt) - kappa Kf + alpha sum_{k=0..k_max} c_k n(t - k dt)
 *   n_hist  device, (k_max+1) x 2N, row k = n(t - k dt) (k_max >= 1 needs two rows)
 *   Kf      device 2N: the kernel applied to the residual q[n(t)] - n(t)
 *   kappa   dt^2 omega^2;  alpha, c (device, k_max+1): dissipation coefficients
 *   n_new   device 2N output (must not overlap n_hist)
 * The paper takes kappa, alpha and c_k from earlier work; they are inputs here.
 */
kk_status kk_xlbomd_update(kk_handle h, const double *n_hist, int k_max, const double *Kf, double kappa,
                           double alpha, const double *c, double *n_new);

/*
 * krylov_kernel_adjoint -- reverse-mode derivative of the rank-m kernel result
 * x = K delta of krylov_kernel_apply (Sec. II.G), for a scalar L(x) whose
 * gradient x_bar = dL/dx the caller supplies (2 x for L = ||K delta||^2).
 *   delta, m, K0   as for krylov_kernel_apply (K0 NULL means -I)
 *   Kdelta_bar     device 2N: x_bar
 *   reuse_forward  0: run the Krylov expansion again first (and write x to
 *                  Kdelta if it is not NULL); 1: use the expansion the last
 *                  krylov_kernel_apply(_adaptive) on this handle left, which
 *                  must have had the same delta, m and K0 (m and K0 are
 *                  checked, KK_EINVAL otherwise; any kk_prepare invalidates it)
 * Outputs (device, caller-owned, overwritten):
 *   delta_bar      2N: dL/d delta
 *   gamma_bar      N x N: dL/d gamma_IJ through the response potentials
 *                  u = gamma v_q +/- W v_m only (not symmetrized: dL = sum_IJ
 *                  gamma_bar_IJ d gamma_IJ)
 *   W_bar          1 double: dL/dW through the response potentials only
 *   H_bar_up, H_bar_dn  Nb x Nb each, or both NULL: dL/dH^sigma with respect to the spin
 *                  Hamiltonians of the prepared expansion point (the H whose
 *                  Z^T H Z has the eigenpairs given to kk_prepare), through the
 *                  levels, the eigenvectors, the occupations and the shared mu
 *                  (Sec. II.C). Symmetric: dL = sum_ij H_bar_ij dH_ij for every
 *                  symmetric dH. A caller that builds gamma, W and H^sigma from
 *                  other parameters (U, W, H0, n) chains through its own
 *                  construction; the expansion-point dependence on gamma and W
 *                  (through H^sigma) is left to that chain.
 * The per-direction response matrices are recomputed in the reverse sweep,
 * never stored. Levels closer than 1e-3 kT (exact degeneracies included) are
 * handled through second divided differences of the Fermi function. With a
 * breakdown (rank r < m) the rank-r expansion is differentiated and
 * KK_BREAKDOWN is returned.
 * Cost and precision. With H_bar_up = H_bar_dn = NULL only delta_bar,
 * gamma_bar and W_bar are formed: one transposed response per direction (m
 * responses, like the forward), in the handle's precision, no workspace beyond
 * O(N m). With the H gradients the reverse sweep runs its transforms in FP64
 * on any handle (about 2.5x the forward's FP64 work; 12 padded Nb^2 FP64
 * matrices of workspace, allocated on first use and kept by the handle): the
 * expansion-point derivative divides commutators of products by level gaps,
 * which turns the ~1e-7 error of split-precision products into ~1e-4. On a
 * KK_MIXED_F16 handle the forward expansion (when recomputed) is split
 * precision, so the gradient is that of the split forward map (~1e-7 from the
 * FP64 one). Synchronizes once (to read the rank) and again if info is not NULL.
 */
kk_status krylov_kernel_adjoint(kk_handle h, const double *delta, int m, const double *K0,
                                const double *Kdelta_bar, int reuse_forward, double *Kdelta,
                                double *delta_bar, double *gamma_bar, double *W_bar,
                                double *H_bar_up, double *H_bar_dn, kk_info *info);

/*
 * Batched form: many independent systems (e.g. uneven Fe clusters) updated
 * together. Every step of the Krylov loop is one launch for all systems (the
 * two transforms are persistent kernels over a global tile list sorted by
 * cost); the whole rank-m update is captured once into a hipGraph on the
 * batch's private stream and replayed, ordered after the caller's stream by
 * events. The first update autotunes the tile shape per system size (64 x 64
 * tiles below a threshold, the single-system shape above) and the number of
 * persistent workgroups per CU by timing every candidate on the batch itself.
 */
typedef struct kk_batch_s *kk_batch;

/* Create a batch ordered after hip_stream (a hipStream_t; NULL = the null stream). */
kk_status kk_batch_create(kk_batch *b, void *hip_stream);

/* Release the batch, its systems and its graph (synchronizes). */
kk_status kk_batch_destroy(kk_batch b);

/*
 * kk_batch_prepare -- kk_prepare for each of n_systems systems (1..4096).
 * Every argument is a HOST array of length n_systems; entries of the pointer
 * arrays are what kk_prepare takes for that system (atom_offsets[i] a host
 * array, the matrices and vectors device arrays). Synchronizes. Replaces any
 * previous preparation of the batch (and its tuning and graph).
 */
kk_status kk_batch_prepare(kk_batch b, int n_systems, const int *n_atoms, const int *const *atom_offsets,
                           const double *const *S, const double *const *Z, const double *const *Q_up,
                           const double *const *Q_dn, const double *const *eps_up, const double *const *eps_dn,
                           const double *const *gamma, const double *W, const double *kT,
                           const double *n_electrons, int precision);

/*
 * krylov_kernel_apply_batch -- krylov_kernel_apply with K0 = -I for every
 * system of the batch. delta and Kdelta are HOST arrays of n_systems device
 * pointers (2 N_i doubles each); 1 <= m <= min(2 N_i, 64). info, if non-NULL,
 * is a HOST array of n_systems entries and makes the call synchronize; the
 * return value is then KK_ESINGULAR or KK_BREAKDOWN if any system reports it.
 * The first call (and the first after kk_batch_prepare) runs the autotuner;
 * a call with a different m captures a new graph.
 */
kk_status krylov_kernel_apply_batch(kk_batch b, const double *const *delta, int m, double *const *Kdelta,
                                    kk_info *info);

/* Tuning chosen by the autotuner (or set by kk_batch_set_tuning): the largest
 * padded size that uses 64 x 64 tiles (0 = none), persistent workgroups per
 * CU, and the fastest update's time in milliseconds (0 when set by hand). */
kk_status kk_batch_tuning(kk_batch b, int *small_np_max, int *workgroups_per_cu, double *update_ms);

/*
 * kk_batch_set_tuning -- fix the tuning instead of letting the first update
 * autotune: systems whose padded size is <= small_np_max (>= 0; 0 = none,
 * a value above every system's = all) take the 64 x 64 tile class, the rest
 * the large one; workgroups_per_cu (1..8) persistent workgroups per CU. Valid
 * after kk_batch_prepare (which resets it); drops any captured graph, so the
 * next update captures anew. For reproducible timings and for tests that must
 * reach each tile class. Synchronizes the batch's stream.
 */
kk_status kk_batch_set_tuning(kk_batch b, int small_np_max, int workgroups_per_cu);

/* Message of the last failing call on this thread ("" if none). */
const char *kk_last_error(void);

/*
 * Kernel timing for measurement. When enabled, the library records HIP events
 * on its stream around each dense transform step of a single-system handle
 * (kernel_id 0: the forward eigenbasis transform with the Fermi Hadamard
 * product, one kernel or the full-tile product followed by its symmetrizing
 * pass; 1: back-transform with the Mulliken projection; 2: the forward
 * transform of the reverse pass, which also writes X; 3: the reverse pass's
 * accumulation of Y0_b Xa + Y0_a Xb). kk_profile_read synchronizes and returns
 * the summed milliseconds and step count since the last reset. At most 8192
 * steps are recorded between resets.
 */
kk_status kk_profile_enable(kk_handle h, int enable);
kk_status kk_profile_reset(kk_handle h);
kk_status kk_profile_read(kk_handle h, int kernel_id, double *total_ms, int *launches);

#ifdef __cplusplus
}
#endif

#endif /* KRYLOV_KERNEL_H */
