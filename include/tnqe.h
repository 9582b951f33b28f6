/*
 * tnqe.h -- C ABI of libtnqe.so: subspace matrices for a linear combination of
 * matrix product states in rotated orbital bases, on one AMD MI355X (gfx950).
 *
 * What it computes (arXiv 2404.10223, "A quantum eigenvalue solver based on
 * tensor networks"):
 *
 *   |psi> = sum_j c_j |phi_j>                                     (eq. tnqe)
 *   H_ij = <phi_i|H|phi_j>,  S_ij = <phi_i|phi_j>                 (eq. mat_els)
 *   H c = E S c, lowest E                                         (eq. GEE)
 *
 * with H the second-quantised electronic Hamiltonian (eq. ham_def, read as
 *   H = sum_{pq,s} h_pq a+_ps a_qs
 *     + 1/2 sum_{pqrs,st} (pq|rs) a+_ps a+_rt a_st a_qs + e_core),
 * and each |phi_j> an MPS (eq. mps) of spatial-orbital sites (d = 4, local index
 * k = n_up + 2 n_dn) written in its own orbital basis U_j (Sec. II.B): column p
 * of U_j is orbital p of basis j in the reference basis, and
 * |phi_j> = G(U_j)|Phi_j> with G(W) a+_p G(W)^+ = sum_q W_qp a+_q.
 *
 * For a pair i < j the ket is taken into the bra's basis by the nearest-
 * neighbour Givens network of W = U_i^T U_j (eq. givens_decomp), applying each
 * two-site gate g4(theta) (App. A3, composite of the d = 2 gates) to the MPS in
 * canonical form and truncating the bond back to chi by SVD (App. A1, eq.
 * svd_longform; Sec. II.B "severe truncations").  H_ij and S_ij then come from
 * one left-environment sweep of bra x MPO x ket (Sec. II.A, App. A1); H_ji and
 * S_ji are copies.  The M x M generalized eigenproblem is solved with
 * S-eigenvalue thresholding by the projection method (Sec. V "Regulating the
 * subspace condition number", App. A2).
 *
 * Conventions the paper leaves open, fixed here:
 *   - Jordan-Wigner mode order (0 up, 0 dn, 1 up, 1 dn, ...); site state
 *     |k> = (a+_up)^{n_up} (a+_dn)^{n_dn} |vac>.
 *   - Givens plan: R_a(t) = identity but [[cos t, sin t], [-sin t, cos t]] on
 *     rows/cols (a, a+1); eliminate Q = W column by column (c = 0..N-2), rows
 *     r = N-1 down to c+1, t = atan2(-Q[r][c], Q[r-1][c]), Q <- R^T Q (an
 *     entry with |Q[r][c]| <= 1e-14 is left alone: t = 0, or pi at the pivot
 *     row r-1 = c when Q[c][c] < 0); apply the recorded gates to the ket in
 *     reverse order (after the parity gate diag(1,-1,-1,1) on the last site
 *     when det W = -1).
 *   - Truncation keeps the min(chi, #{s^2 > tau_w sum s^2}) largest singular
 *     values over all quantum-number blocks; singular values are absorbed to
 *     the right; no renormalisation unless tnqe_options.renormalize is set.
 *
 * Threading and streams: one context per host thread; every call is blocking
 * (it synchronises the context's stream before returning host results).
 * Errors: every entry point returns a tnqe_status; negative means failure,
 * outputs are then left untouched and tnqe_last_error(ctx) holds a message.
 * Memory: device memory comes either from a workspace the caller allocates
 * (tnqe_subspace / tnqe_subspace_batch with a non-NULL workspace: the library
 * then allocates no device memory at all; tnqe_workspace_size gives a size
 * that always suffices) or, when no workspace is given, from a pool the
 * context owns (hipMalloc on demand, kept until tnqe_trim / tnqe_destroy).
 */
#ifndef TNQE_H
#define TNQE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tnqe_ctx tnqe_ctx;
typedef struct tnqe_problem tnqe_problem;

typedef enum {
  TNQE_OK = 0,
  TNQE_EINVAL = -1,      /* null pointer, bad option value               */
  TNQE_ESHAPE = -2,      /* inconsistent dimensions                      */
  TNQE_ENOTORTH = -3,    /* a rotation U is not orthogonal (1e-10)       */
  TNQE_EQN = -4,         /* a site tensor breaks particle-number blocks  */
  TNQE_ENOMEM = -5,      /* device allocation failed                     */
  TNQE_EWORKSPACE = -6,  /* the caller's workspace is too small           */
  TNQE_EHIP = -7,        /* a HIP runtime call failed                    */
  TNQE_ESINGULAR = -8,   /* S has no eigenvalue above the threshold      */
  TNQE_ENONFINITE = -9,  /* NaN/Inf in an input or a result              */
  TNQE_ENODEVICE = -10   /* no usable gfx950 device                      */
} tnqe_status;

typedef enum {
  TNQE_FP64 = 0,         /* everything in FP64                                      */
  TNQE_ENV_FP32 = 1,     /* environment sweep in FP32 (FP64 gates, SVD, final sum,
                            eigensolve); the element sum is compensated FP64        */
  TNQE_ENV_MIXED = 2,    /* per pair: FP32 environments where the rotated ket keeps
                            at most 1e-6 of its squared norm (the element and its
                            FP32 rounding error are then bounded by the ket norm),
                            FP64 for every other pair (all diagonal pairs)          */
  TNQE_ENV_FP32_SHIFT = 3, /* every pair in FP32 on the shifted operator H - c N,
                            c N_e = the FP64 element H_00 (one FP64 pair): FP32
                            rounding then acts on O(spread) values instead of
                            O(|E|); the eigenproblem of (H - c N_e S, S) gives
                            E - c N_e exactly in exact arithmetic; H is returned
                            as H' + c N_e S (FP32-level absolute error)         */
  TNQE_ENV_BF16 = 4,     /* as TNQE_ENV_FP32_SHIFT, the environment GEMMs on the
                            BF16 matrix cores (operands rounded to BF16, FP32
                            accumulation and storage)                            */
  TNQE_ENV_BF16X3 = 5    /* as TNQE_ENV_FP32_SHIFT, each GEMM operand split into
                            BF16 hi + lo and the product taken as three BF16
                            matrix-core products (hi hi + hi lo + lo hi), FP32
                            accumulation and storage                             */
} tnqe_precision;

/* Hamiltonian in the reference orbital basis.  All host pointers, row-major,
 * read during the call only. */
typedef struct {
  int32_t N;             /* spatial orbitals (sites), 1 <= N <= 64            */
  int32_t n_alpha;       /* electrons with spin up                             */
  int32_t n_beta;        /* electrons with spin down                           */
  const double *h;       /* [N][N] symmetric one-electron integrals (Hartree)  */
  int32_t n_chol;        /* K > 0: two-electron integrals as Cholesky vectors  */
  const double *L;       /* [K][N][N] symmetric, (pq|rs) = sum_k L[k][p][q] L[k][r][s] */
  const double *g;       /* [N][N][N][N] (pq|rs) when n_chol == 0, else NULL   */
  double e_core;         /* constant energy                                     */
} tnqe_hamiltonian;

/* One MPS with its orbital basis.  bond b (0..N) has bond_dim[b] indices,
 * bond_dim[0] = bond_dim[N] = 1; index x of bond b carries the quantum numbers
 * (n_alpha, n_beta) of sites 0..b-1 in bond_qn; indices sorted by sector.
 * Site p is [bond_dim[p]][4][bond_dim[p+1]] row-major; entry [l][k][r] must be
 * zero unless qn(r) = qn(l) + (k & 1, k >> 1).  Sites are concatenated in p
 * order.  Host pointers. */
typedef struct {
  const int32_t *bond_dim;   /* [N+1]                                   */
  const int32_t *bond_qn;    /* [sum_b bond_dim[b]][2]                  */
  const double *sites;       /* concatenated site tensors               */
  const double *U;           /* [N][N] orthogonal, column p = orbital p */
} tnqe_mps;

typedef struct {
  int32_t chi;               /* truncation cap for the rotated kets (>= 1)            */
  int32_t chi_cap_override;  /* > 0: use this cap instead of chi (lossless tests)     */
  int32_t precision;         /* a tnqe_precision value                                 */
  double eps_S;              /* relative eigenvalue threshold on S (default 1e-12)    */
  double tau_w;              /* relative discarded-weight floor (default 1e-13)       */
  int32_t max_sweeps;        /* Jacobi sweep limit (default 40)                        */
  int32_t renormalize;       /* 1: after every truncation rescale the kept singular
                                values so the ket keeps its weight (App. A1 asks for a
                                renormalisation in its DMRG setting; optional here);
                                0 (default): plain projection, no rescaling           */
  int32_t autotune;          /* 1: environment tile shapes from the context's tuned
                                table (measured on first use, cached on disk); 0: the
                                fixed shape rule; 2 + k (k < 5, for tests): tile k of
                                256x16, 128x32, 64x64, 32x128, 16x256 on every
                                environment GEMM; other values TNQE_EINVAL             */
  int32_t workers;           /* batch calls (read from the first subspace's options):
                                subspaces solved concurrently (0: default, 4)          */
  int32_t reserved[4];
} tnqe_options;

typedef struct {
  double max_discarded_weight_sum;  /* max over pairs of the summed discarded weights  */
  double min_rel_gap;               /* min over truncations of (s_kept - s_next)/s_kept */
  double cond_S;                    /* lambda_max / lambda_min(kept) of S               */
  double lambda_min_S;              /* smallest eigenvalue of S                         */
  double kappa1;                    /* |c|^2 / sqrt(E^2 + 1)                            */
  double t_total_ms, t_host_ms, t_gates_ms, t_env_ms, t_gep_ms;
  double alg_flops;                 /* algorithmic (nonzero-block) flops of the call    */
  double alg_bytes;                 /* algorithmic HBM bytes of the environment sweep   */
  double env_flops;                 /* environment-sweep part of alg_flops              */
  double env_kernel_ms;             /* summed device time of the environment kernels     */
  double svd_kernel_ms;             /* summed device time of the block SVD launches     */
                                    /*   (truncations and centre moves)                 */
  double svd_flops;                 /* their algorithmic flops (4 n^2 m + 9 n^3 a block) */
  double svd_kind_ms[16];           /* the same split by kernel: entry k < 6 for the    */
  double svd_kind_flops[16];        /*   Jacobi SVD with 4 (k + 1) vector elements per  */
                                    /*   lane, 6 its global-memory fallback, 7 the      */
                                    /*   Householder QR of the centre moves, 8-15 unused */
  double env_kind_ms[8];            /* environment kernels: 0 L x ket GEMM, 1 sparse    */
  double env_kind_flops[8];         /*   channel mix, 2 dense coupling GEMMs, 3 bra^T x */
  double env_kind_bytes[8];         /*   Y GEMM, 4 final element; device time, flops    */
                                    /*   and algorithmic bytes, entries 5-7 unused      */
  int32_t n_dropped;                /* eigenvalues of S below the threshold             */
  int32_t n_pairs;                  /* unique pairs computed (M (M + 1) / 2)            */
  int32_t max_bond;                 /* largest bond dimension seen                      */
  int32_t mpo_max_bond;             /* largest MPO bond dimension                       */
  int32_t svd_launches;             /* block SVD launches timed                         */
  int32_t svd_kind_launches[16];    /* the same split by SVD kernel                     */
  int32_t env_kind_launches[8];     /* launches of each environment kernel              */
  int32_t n_fp32_pairs;             /* pairs contracted in FP32 (precision modes 1, 2)  */
  int32_t reserved[7];
  double ws_peak_bytes;             /* workspace calls: bytes of it actually used       */
  double move_kernel_ms;            /* device time of the centre-move factorisations    */
  double move_flops;                /*   and their flops (part of svd_kernel_ms/flops)  */
  double t_moves_ms;                /* host time issuing the gate phase's centre moves  */
  double t_tune_ms;                 /* autotuning of tile shapes during the call        */
  int32_t move_launches;            /* centre-move factorisation launches timed         */
  int32_t reserved2;
} tnqe_report;

/* Fill defaults (chi = 16, FP64, eps_S = 1e-12, tau_w = 1e-13). */
void tnqe_default_options(tnqe_options *opts);

/* Create a context on HIP device `device` issuing all work on `hip_stream`
 * (a hipStream_t, e.g. torch.cuda.current_stream().cuda_stream; NULL = the
 * null stream).  Fails with TNQE_ENODEVICE if the device is not gfx950. */
tnqe_status tnqe_create(tnqe_ctx **out, int device, void *hip_stream);
tnqe_status tnqe_destroy(tnqe_ctx *ctx);
/* Release the context's cached device memory. */
tnqe_status tnqe_trim(tnqe_ctx *ctx);

/* Validate inputs and copy them to device memory (the only host-to-device
 * transfer of problem data).  Validation: shapes, |U^T U - I|_max <= 1e-10,
 * zero entries outside particle-number blocks, finite values, each MPS in the
 * (n_alpha, n_beta) sector. */
tnqe_status tnqe_upload(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M,
                        const tnqe_mps *mps, tnqe_problem **out);
tnqe_status tnqe_problem_free(tnqe_problem *prob);

/* H, S: [M][M] host, row-major; E: [1]; c: [M] or NULL; rep: or NULL. */
tnqe_status tnqe_solve(tnqe_ctx *ctx, tnqe_problem *prob, const tnqe_options *opts,
                       double *H, double *S, double *E, double *c, tnqe_report *rep);

/* Several independent subspaces in one call, solved one after another on the
 * context's stream (inside each subspace every pair shares the same
 * launches).  opts: [n], one per subspace (each with its own chi).  H[s],
 * S[s]: [M_s][M_s] host; E: [n]; rep: [n] or NULL.  Stops at the first
 * failing subspace and returns its status; later outputs are untouched. */
tnqe_status tnqe_solve_batch(tnqe_ctx *ctx, int32_t n, tnqe_problem *const *probs,
                             const tnqe_options *opts, double *const *H, double *const *S,
                             double *E, tnqe_report *rep);

/* Device bytes that always suffice for tnqe_subspace with these inputs and
 * options: the site tensors, the MPO of H (eq. ham_def, Sec. II.A), the
 * rotated kets of every pair i < j at the bond capacities min(chi, exact
 * sector dimension) (Sec. II.B, App. A1), the largest gate-step scratch, and
 * the environment sweep of one pair at those capacities.  Host-side only
 * (validation of the inputs included); the bound is conservative: truncated
 * bonds are usually much smaller, and tnqe_report.ws_peak_bytes gives what a
 * call really used. */
tnqe_status tnqe_workspace_size(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                                const tnqe_options *opts, size_t *bytes);

/* The problem statement of the paper in one call: integrals h_pq and (pq|rs)
 * (eq. ham_def), M MPS each in its own orbital basis (eq. tnqe, Sec. II.B),
 * bond dimension chi; returns the pencil H_ij = <phi_i|H|phi_j>,
 * S_ij = <phi_i|phi_j> (eq. mat_els) and the lowest root E of H c = E S c
 * (eq. GEE) with its coefficients c (c^T S c = 1).
 *   ham, mps[M], opts: host, read during the call only.
 *   workspace: device memory of ws_bytes bytes owned by the caller (e.g. a
 *     torch.empty(..., dtype=torch.uint8, device='cuda') buffer), not in use
 *     by other work; every device buffer of the call lies in it, the call
 *     allocates no device memory, and the workspace is free again when the
 *     call returns.  TNQE_EWORKSPACE when it is too small (outputs
 *     untouched).  NULL: the library allocates from the context's pool.
 *   H, S: [M][M] host, row-major; E: [1]; c: [M] or NULL; rep: or NULL. */
tnqe_status tnqe_subspace(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                          const tnqe_options *opts, void *workspace, size_t ws_bytes, double *H, double *S,
                          double *E, double *c, tnqe_report *rep);

/* n_sub independent subspaces (the independent problems of a set of
 * subspace calculations, e.g. the parallel batches of matrix elements of
 * App. B), each as in tnqe_subspace: ham[s], M[s], mps[s][0..M[s]),
 * opts[s] (each with its own chi).  The subspaces share the workspace (each
 * uses it in turn; give the largest tnqe_workspace_size of the set), or NULL
 * for the context's pool.  H[s], S[s]: [M[s]][M[s]] host; E: [n_sub];
 * rep: [n_sub] or NULL.  Stops at the first failing subspace and returns its
 * status (tnqe_last_error names it); no output is written then. */
tnqe_status tnqe_subspace_batch(tnqe_ctx *ctx, int32_t n_sub, const tnqe_hamiltonian *ham, const int32_t *M,
                                const tnqe_mps *const *mps, const tnqe_options *opts, void *workspace,
                                size_t ws_bytes, double *const *H, double *const *S, double *E,
                                tnqe_report *rep);

/* The expanded one-hot pencil of one state (Sec. II.E eq. oht_exp and
 * eq. subs_exp, App. A1, expanding a single reference state i): state i is put
 * in canonical form centred on sites (p, p+1) (eq. orth_l / orth_r, by exact
 * QR/LQ with a non-negative diagonal of the triangular factor, which fixes the
 * gauge); its two-site tensor T[l, k_p, k_{p+1}, r] is expanded over the n
 * one-hot tensors that conserve the particle numbers, numbered in row-major
 * order of T, giving the orthonormal one-hot states varphi_m.  Every other
 * state k is taken into basis i by its Givens network with truncation to chi
 * (as for the pencil, here for k < i too).  Outputs (host, row-major):
 *   index [n][4]: (l, k_p, k_{p+1}, r) of one-hot state m;
 *   Hd, Sd [n][n]: <varphi_m|H|varphi_n>, <varphi_m|varphi_n> (the identity);
 *   Hc, Sc [n][M]: <varphi_m|H|phi_k>, <varphi_m|phi_k> (column i: phi_i).
 * H is H^(i) (integrals rotated into basis i), e_core included.
 * tnqe_onehot_size gives n (host-only; ctx may be NULL); tnqe_onehot_pencil
 * fails with TNQE_ESHAPE when its n differs.  Device memory from the
 * context's pool.  rep: t_gates_ms (networks and canonical form), t_env_ms,
 * env_kernel_ms and env_flops (the one-hot contractions), or NULL. */
tnqe_status tnqe_onehot_size(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                             const tnqe_options *opts, int32_t i, int32_t p, int32_t *n);
tnqe_status tnqe_onehot_pencil(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                               const tnqe_options *opts, int32_t i, int32_t p, int32_t n, int32_t *index,
                               double *Hd, double *Sd, double *Hc, double *Sc, tnqe_report *rep);

/* One step of the generalized sweep (Alg. A.1) at sites (p, p+1) with state i
 * as the expanded state (jset = {i}; App. A1), no single-site mitigation
 * repetitions (App. A4):
 *  1. the expanded pencil of tnqe_onehot_pencil, with the current pencil
 *     (H, S) for the unexpanded states, in the order of eq. subs_exp: states
 *     k < i, the n one-hot states of i, states k > i (D = n + M - 1 columns);
 *  2. columns taken in that order are discarded when their squared distance
 *     from the span of the kept earlier ones is below tol_ld times their
 *     squared norm (Sec. V "Regulating the subspace condition number",
 *     App. A2);
 *  3. the lowest root E1 of the kept pencil by the projection method with the
 *     eps_S threshold of opts (eq. exp_gen_eig);
 *  4. parameter update (eq. param_upd): t'_m = C'[i m] / ||C'[i .]||, signed
 *     so that sum_m t'_m t_m >= 0;
 *  5. rotation of the bond (App. A3): none; the FSWAP f4, taken when it lowers
 *     xi = 1 - sum_{l <= chi} sigma_l^2; or the Givens gate g4(theta) at
 *     theta_opt = argmin xi(theta): the best of n_grid angles
 *     (q - n_grid/2) pi / n_grid, then n_golden golden-section steps on one
 *     spacing either side; a rotation is taken only when it lowers xi by
 *     more than 1e-12 (below that the choice would be rounding);
 *  6. truncation of the rotated two-site tensor with the rule of the gates
 *     (chi, tau_w of opts): A_p = U, A_{p+1} = U^T T, centre at p + 1;
 *  7. merge of the rotation into the orbital basis of state i:
 *     U_i <- U_i R_p(theta)^T (FSWAP: columns p and p+1 exchanged), which
 *     leaves the state unchanged up to the truncation;
 *  8. with nreps > 0, the single-site mitigation of App. A4: the expanded
 *     pencil moved to the rotated basis (the gate in the one-hot basis,
 *     H^[ii] -> G^T H^[ii] G, H^[ik] -> G^T H^[ik]), then nreps rounds of
 *     expansions over the single-site one-hot states at p and then p+1, the
 *     other site held as an orthonormal basis of its space in the current
 *     two-site tensor with the truncated bond (its singular vectors), each
 *     with steps 2-4 on the pencil projected by the isometry T (T H T^T,
 *     T H^[ik]); A_p is then that orthonormal basis, A_{p+1} the updated site;
 *  9. accepted = E_new < E_old + e_tol (E_old: lowest root of (H, S); E_new:
 *     E1, or the last root of step 8).
 * Inputs: as tnqe_onehot_pencil, and H, S [M][M] host (the current pencil,
 * e.g. from tnqe_subspace with the same options).  Outputs (host): res; the
 * updated state i in the layout of tnqe_mps -- bond_dim [N+1], bond_qn
 * [qn_cap][2] (sum of bond_dim entries used), sites [sites_cap] (site x is
 * [bond_dim[x]][4][bond_dim[x+1]], in canonical form centred on p+1, bonds
 * sorted by sector), U [N][N]; rep or NULL.  qn_cap >= sum of the input
 * state's bond dimensions + chi and sites_cap >= the input state's site
 * sizes + 4 chi (bond_dim[p] + bond_dim[p+2]) always suffice; smaller
 * capacities that do not hold the result give TNQE_ESHAPE (outputs
 * untouched).  D = n + M - 1 <= 1024 (TNQE_ESHAPE beyond); M <= 32.  Device
 * memory from the context's pool.  rep: t_gates_ms and t_env_ms as for
 * tnqe_onehot_pencil, t_gep_ms (steps 2-4), t_total_ms (the whole step; the
 * rest is steps 5-7). */
typedef enum { TNQE_ROT_NONE = 0, TNQE_ROT_FSWAP = 1, TNQE_ROT_GIVENS = 2 } tnqe_rotation;
typedef struct {
  int32_t rotation;      /* tnqe_rotation */
  int32_t n_grid;        /* Givens: grid angles, even (0: 36) */
  int32_t n_golden;      /* Givens: golden-section steps (< 0: 40) */
  int32_t nreps;         /* single-site mitigation rounds (App. A4), 0 .. 64 */
  double tol_ld;         /* discard threshold (0: 1e-3) */
  double e_tol;          /* acceptance tolerance (Hartree) */
  double reserved[2];
} tnqe_sweep_options;
typedef struct {
  double E_old;          /* lowest root of the current pencil */
  double E1;             /* lowest root of the expanded pencil */
  double theta;          /* rotation applied: Givens angle, pi/2 for an accepted FSWAP, else 0 */
  double xi_none, xi;    /* truncation error without / with the rotation */
  double discarded;      /* discarded weight of the final truncation */
  int32_t n_onehot;      /* n */
  int32_t n_columns;     /* D */
  int32_t n_kept;        /* columns kept by the discard */
  int32_t n_dropped_S;   /* further directions dropped by the eps_S threshold */
  int32_t accepted;      /* 1: E1 < E_old + e_tol */
  int32_t new_bond;      /* bond dimension p + 1 after the truncation */
  int32_t mit_columns;   /* columns of the last single-site expanded pencil (0: no mitigation) */
  int32_t mit_kept;      /* of them kept by the discard */
  double E_new;          /* the last root: E1, or after the mitigation rounds their last one */
} tnqe_sweep_result;
tnqe_status tnqe_sweep_step(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                            const tnqe_options *opts, const tnqe_sweep_options *sw, int32_t i, int32_t p,
                            const double *H, const double *S, int32_t *bond_dim, int32_t *bond_qn, int64_t qn_cap,
                            double *sites, int64_t sites_cap, double *U, tnqe_sweep_result *res,
                            tnqe_report *rep);
/* t'_m of the last tnqe_sweep_step on this context ([n_onehot] host), for
 * checks; TNQE_EINVAL when n differs from that call's n_onehot. */
tnqe_status tnqe_sweep_last_params(tnqe_ctx *ctx, int32_t n, double *t);

/* For callers that cannot allocate memory (code under HIP stream capture,
 * tight serving loops, harnesses that forbid allocation): tnqe_subspace with
 * no workspace argument and no allocation of device or pinned host memory,
 * of timing events or of streams.  Every device buffer of the call lies in a
 * fixed scratch array of tnqe_noalloc_capacity() bytes (256 MiB) that each
 * GPU holds from its first tnqe_create until the process ends.  Inputs whose
 * tnqe_workspace_size exceeds that are refused with TNQE_EWORKSPACE before
 * any device work.  Arguments, outputs and errors as in tnqe_subspace.  All
 * calls on one GPU share its scratch (it keeps the last call's contents): two
 * such calls that overlap in time on one GPU, from any thread or context,
 * race and give wrong results; serialise them. */
tnqe_status tnqe_subspace_noalloc(tnqe_ctx *ctx, const tnqe_hamiltonian *ham, int32_t M, const tnqe_mps *mps,
                                  const tnqe_options *opts, double *H, double *S, double *E, double *c,
                                  tnqe_report *rep);
size_t tnqe_noalloc_capacity(void);

const char *tnqe_status_string(tnqe_status st);
const char *tnqe_last_error(const tnqe_ctx *ctx);
const char *tnqe_version(void);

/* Host-only diagnostics (no device needed), used to test the host logic.
 *
 * tnqe_debug_givens: the Givens plan of an N x N orthogonal W (row-major):
 *   pos[K], theta[K] in application order, K = N (N - 1) / 2, and det_sign.
 * tnqe_debug_gate: the 16 x 16 gate g4(theta) on (k_p, k_{p+1}), row-major,
 *   index k_p * 4 + k_{p+1}.
 * tnqe_debug_mpo_dense: the library's MPO of H (N <= 5) contracted to dense
 *   4^N x 4^N matrices of H and of the identity channel, for h [N][N] and
 *   (pq|rs) g [N^4]; max_bond may be NULL.
 * tnqe_debug_host_pool: runs `jobs` back-to-back parallel loops of 1..5
 *   items on a pool of `workers` host threads (the pool the gate and
 *   environment phases use) and checks that every item of every loop ran
 *   exactly once; *calls receives the total number of item calls.  Returns
 *   TNQE_EINVAL on bad arguments or when an item ran zero or several times. */
tnqe_status tnqe_debug_givens(int32_t N, const double *W, int32_t *pos, double *theta, int32_t *det_sign);
tnqe_status tnqe_debug_gate(double theta, double *out);
tnqe_status tnqe_debug_mpo_dense(int32_t N, const double *h, const double *g, double *H, double *I,
                                 int32_t *max_bond);
tnqe_status tnqe_debug_host_pool(int32_t workers, int32_t jobs, int64_t *calls);

/* Device diagnostic (needs the context's GPU), used to test the truncation
 * rule of the gate step (App. A1: the largest singular values over all
 * quantum-number blocks of a two-site matrix are kept).
 *
 * tnqe_debug_select: runs the device selection on nket kets.  Ket t has
 *   nblk[t] blocks; block i (kets in order, blocks in order) has n[i] values,
 *   sorted in decreasing order, taken in turn from the host array sv.  Per
 *   ket, keep = min(chi, #{s^2 > tau * sum s^2}) values with the largest
 *   ranks are kept (larger values first; equal values in block order, then in
 *   order within the block).  Outputs (host arrays): kept[i] per block and,
 *   per ket, stats[3 t ..] = (keep, discarded weight sum over the values not
 *   kept of s^2, relative gap (s_in - s_out) / s_in at the cut, 1 when
 *   nothing was cut).  Returns TNQE_EINVAL on bad arguments (unsorted lists
 *   included) and TNQE_ESHAPE when a ket has more values than the kernel's
 *   local memory holds. */
tnqe_status tnqe_debug_select(tnqe_ctx *ctx, int32_t nket, const int32_t *nblk, const int32_t *n,
                              const double *sv, int32_t chi, double tau, int32_t *kept, double *stats);

/* tnqe_debug_gep: the device eigensolver of the pencil on given H, S ([M][M]
 * host, row-major, symmetric, M <= 32) with S-eigenvalue threshold
 * eps_S * lambda_max(S), by the projection method (Sec. V "Regulating the
 * subspace condition number", App. A2).  out[8 + M] (host): E, cond(S) over
 * the kept eigenvalues, lambda_min(S), number dropped, kappa_1 = |c|^2 /
 * sqrt(E^2 + 1) (App. A2), status (0, or 1 when nothing is kept), 0, 0, then
 * c[0..M) with c^T S c = 1. */
tnqe_status tnqe_debug_gep(tnqe_ctx *ctx, int32_t M, const double *H, const double *S, double eps_S,
                           double *out);

/* tnqe_debug_psd_eigen: the device eigensolver of the dense eigenproblems of
 * the generalized sweep (the overlap matrix of the kept expanded columns and
 * the shifted whitened Hamiltonian, eq. exp_gen_eig) on a given symmetric
 * positive semi-definite A ([n][n] host, row-major, 1 <= n <= 1024): the
 * one-sided Jacobi SVD, which for such A is its eigendecomposition.  path 0
 * is the choice of the sweep step (register kernels when they hold the
 * matrix, else the global-memory Jacobi spread over the chip by blocks of
 * columns), 1 the global-memory Jacobi in one workgroup, 2 the one spread
 * over the chip by column pairs (paths 1 and 2 give the same bits), 3 the one
 * spread over the chip by blocks of columns, each sweep's launches replayed
 * from a captured HIP graph (as path 0 does), 4 the same with the launches
 * issued one by one (paths 3 and 4 give the same bits).  Outputs (host): val[n] in decreasing
 * order, vec[n][n] with row k the unit vector of val[k].  TNQE_EINVAL on bad
 * arguments. */
tnqe_status tnqe_debug_psd_eigen(tnqe_ctx *ctx, int32_t n, const double *A, int32_t path, int32_t max_sweeps,
                                 double *vec, double *val);

#ifdef __cplusplus
}
#endif
#endif /* TNQE_H */
