/*
 * splitctm.h -- C ABI of the MI355X (gfx950) split-CTMRG library.
 *
 * The library computes, for an infinite PEPS given by a periodic unit cell of
 * real site tensors A[x][y] (Sec. II A, the coefficient tensor network), the
 * split-CTMRG environment of Sec. II B (Fig. split-transfer-ctmrg: corners
 * C1..C4 and, per edge, a ket and a bra transfer tensor joined by an
 * interlayer bond of dimension chi_I), the projectors of the left move
 * (Fig. proj_plots_green and App. A: green, teal, yellow, red), the energy of
 * a nearest-neighbour Hamiltonian (Sec. III) and its gradient with respect to
 * the site tensors (reverse mode through the whole update, Sec. III).
 *
 * Conventions
 *   - Site tensors: FP64, C order, [Lx][Ly][p][D][D][D][D] with the legs of
 *     each site ordered (physical, up, left, down, right); x = row, y = column.
 *   - Environment tensors of one site, in this order ("packed layout"):
 *       C1[d][r] C2[l][d] C3[u][l] C4[r][u]                   chi_E x chi_E each
 *       T1k[l][s][r] T1b T2k[u][s][d] T2b T3b[r][s][l] T3k T4b[d][s][u] T4k
 *     the first tensor along each edge (T1k, T2k, T3b, T4b) is
 *     [chi_E][D][chi_I], the second (T1b, T2b, T3k, T4k) is [chi_I][D][chi_E];
 *     sites follow in row-major [x][y] order.  FP64, C order.
 *   - All device pointers (A, dA, workspace, env buffers) are owned by the
 *     caller; the library never allocates device memory.  The context object
 *     itself is host memory, released by ctm_destroy.
 *   - All work is ordered on the HIP stream given to ctm_init; calls that
 *     return host scalars synchronise that stream.  One context per stream;
 *     calls on one context are not reentrant.  A context made by ctm_init
 *     also owns one internal stream of default priority (created there,
 *     destroyed by ctm_destroy) on which the Q factors of its QR
 *     decompositions are formed; every such piece of work is joined into the
 *     caller's stream (stream-wait on an event) before the call that issued
 *     it returns, so the caller sees one ordered stream.  ctm_init_static
 *     creates no stream.
 *   - Projector SVDs, truncation, normalisation reductions and the final
 *     energy reduction are always FP64; `contract_prec` sets the precision of
 *     the tensor-network contractions.  The one-sided Jacobi SVD runs to
 *     working accuracy with FP64 contractions and to a relative
 *     off-orthogonality of 1e-10 with FP32, BF16x3 or BF16x6 contractions,
 *     whose own rounding is larger; its singular vectors are orthonormal to
 *     FP64 rounding in every case (the reverse pass needs that).
 *
 * Errors: every call returns a ctm_status.  CTM_EINVAL = bad argument or
 * workspace too small (no side effects); CTM_ENUMERIC = non-finite values or a
 * rank-zero projector matrix; CTM_ENOTCONV = sweep budget exhausted before the
 * tolerance was met (the environment is still valid); CTM_EDEVICE = a HIP
 * runtime error.  ctm_strerror never returns NULL.
 */
#ifndef SPLITCTM_H
#define SPLITCTM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CTM_OK = 0,
  CTM_EINVAL = 1,
  CTM_ENOMEM = 2,
  CTM_EDEVICE = 3,
  CTM_ENOTCONV = 4,
  CTM_ENUMERIC = 5
} ctm_status;

/* Contraction precision: FP64; FP32 (FP32 matrix cores); BF16X3 = FP32
 * operands split as hi + lo in bf16, products lo*hi + hi*lo + hi*hi on the
 * BF16 matrix cores with FP32 accumulation (error ~2^-16 relative per
 * product); BF16X6 = three-way split hi + mid + lo with the six products of
 * total order below 3 (error near FP32 rounding). */
typedef enum { CTM_FP64 = 0, CTM_FP32 = 1, CTM_BF16X3 = 2, CTM_BF16X6 = 3 } ctm_precision;

/* Boundary of ctm_init: IDENTITY = chi_E = 1 corners and transfer tensors
 * that trace the ket and bra virtual legs (independent of A); PRODUCT = every
 * transfer tensor carries a given vector v on its physical-side leg (fixes the
 * boundary configuration, e.g. an ordered Ising boundary). A random start is
 * passed in with ctm_env_import. */
typedef enum { CTM_INIT_IDENTITY = 0, CTM_INIT_PRODUCT = 1 } ctm_init_mode;

/* Projector constructions (bit flags).  APP_A (0): the networks of App. A.
 * ALT_YR: the alternative yellow / red projectors of App. B (Figs.
 * alternativeConstructionYellowProjectors, alternativeConstructionRedProjectors):
 * the yellow networks of App. A, but the physical leg is cut together with
 * (chi_I, D), so M_yellow spans only the (D, chi_I) legs, and red truncates
 * (chi_I, D); no SVD then carries the p factor.  HALF_TEAL: the teal half
 * projectors of App. B (the analogue of half projectors; the paper's network
 * figure has no body): the teal half networks are the left column of the
 * 2-column patch, with their legs towards the right left open, so M_teal is
 * chi_E D^2-dimensional with rank <= chi_E D (chi_E D^2 <= 8192).  The two
 * flags combine. */
typedef enum { CTM_PROJ_APP_A = 0, CTM_PROJ_ALT_YR = 1, CTM_PROJ_HALF_TEAL = 2 } ctm_projector_variant;

typedef struct {
  int Lx, Ly;                  /* unit cell: rows, columns */
  int p, D;                    /* physical and bulk bond dimension */
  int chi_E, chi_I;            /* environment and interlayer bond dimension */
  ctm_precision contract_prec; /* bulk contractions */
  double svd_rel_cutoff;       /* drop singular values below cutoff * s_1 (<= 0: 1e-12) */
  double svd_adj_eps;          /* Lorentzian broadening of the SVD adjoint (<= 0: 1e-12) */
  ctm_init_mode init;
  int projector_variant;       /* ctm_projector_variant flags */
} ctm_config;

typedef struct ctm_ctx ctm_ctx;

/* Bytes of device workspace needed for a context of this configuration.
 * with_grad != 0 reserves what ctm_energy_grad(n_sweeps, ckpt_every) needs. */
ctm_status ctm_workspace_size(const ctm_config* cfg, int with_grad, int n_sweeps, int ckpt_every, size_t* bytes);

/* Create a context for the unit cell {A[x][y]} of Sec. II A (the
 * coefficient tensor network of the iPEPS, one real tensor per site of the
 * periodic cell) and the split environment of Sec. II B with bond dimensions
 * chi_E (environment) and chi_I (interlayer).  Copies A (device, FP64, layout
 * above; the caller keeps ownership) into the workspace, writes the initial
 * environment (boundary_vec_host: length D, PRODUCT only, else NULL) and
 * keeps it as the start environment of ctm_energy_grad.  The workspace
 * (device, ws_bytes >= ctm_workspace_size) belongs to the caller and must
 * outlive the context.  CTM_EINVAL for an invalid configuration, a NULL A or
 * workspace, or a workspace too small for the persistent part; *out is then
 * NULL. */
ctm_status ctm_init(const ctm_config* cfg, const double* A_dev, const double* boundary_vec_host, void* workspace_dev,
                    size_t ws_bytes, void* hip_stream, ctm_ctx** out);

/* Directional sweeps (left, top, right, bottom move; Sec. II B, Eqs.
 * splitCTMRG_C1, splitCTMRG_C4, splitCTMRG_Tket, splitCTMRG_Tbra for the left
 * move, the others by lattice symmetry) until the corner singular values
 * change by less than tol over one sweep (2-norm of the difference of the
 * zero-padded spectra, largest over all corners of the cell) or max_sweeps
 * are done.  tol <= 0 runs exactly max_sweeps.  *delta (optional) = that
 * change over the last sweep run (the spectra of the sweep's start
 * environment are taken first when they are not known).  CTM_ENOTCONV when
 * tol > 0 was not reached (the environment is valid); CTM_ENUMERIC for a
 * non-finite change. */
ctm_status ctm_sweep(ctm_ctx* ctx, int max_sweeps, double tol, int* sweeps_done, double* delta);

/* Projectors of Fig. proj_plots_green (the recipe: the product of the two
 * half networks over the legs to keep, its truncated SVD, and the pair
 * P_T = rho_B U_k S_k^{-1/2}, P_B = rho_T V_k S_k^{-1/2}) for the four
 * colours of App. A.
 * The four projector pairs of the move in `direction` (0 left, 1 top,
 * 2 right, 3 bottom) for the cut below row x / row x of the column holding
 * site [x][y] (in that move's frame), from the current environment, which is
 * not modified.  out_dev (FP64, device) receives, in order, green P_T, P_B
 * [chi_E][D][chi_E], teal P_T, P_B [chi_E][D][chi_E], yellow P_T, P_B
 * [chi_I][D][chi_I] and red P_T, P_B [chi_I][p][D][chi_I] (ALT_YR: yellow
 * [chi_I][D][p][chi_I], red [chi_I][D][chi_I]); columns beyond the
 * kept rank are zero.  trunc_err_host[4] = discarded weight sum_{k>=kept}
 * s_k^2 / sum s_k^2 of green, teal, yellow, red. */
ctm_status ctm_projectors(ctm_ctx* ctx, int direction, int x, int y, double* out_dev, double* trunc_err_host);
size_t ctm_projectors_elems(const ctm_config* cfg);

/* One column of one directional move (Sec. II B: the left move absorbs the
 * columns of the cell one after the other, Eqs. splitCTMRG_C1,
 * splitCTMRG_C4, splitCTMRG_Tket, splitCTMRG_Tbra): in the frame of
 * `direction` (0 left, 1 top, 2 right, 3 bottom, as in ctm_projectors),
 * column y of the cell is absorbed into the left environment of column y+1,
 * whose C1, T4k, T4b, C4 (in that frame) are replaced in the current
 * environment; nothing else changes.  A sweep is the four moves, each over
 * every column in order.  For checks of a single step at full size.
 * CTM_EINVAL for a direction outside 0..3 or a column outside the frame's
 * cell. */
ctm_status ctm_move_column(ctm_ctx* ctx, int direction, int y);

/* Sec. III: the expectation value of a nearest-neighbour Hamiltonian from
 * the converged environment, each bond's two-site reduced density matrix
 * being the 2-row patch of Fig. proj_plots_green with both physical legs
 * open.  The final reduction is FP64 on the GPU.
 * Energy per site of the nearest-neighbour Hamiltonian h (host, FP64,
 * p^2 x p^2 row-major, rows (s1 s2) bra, columns (s1 s2) ket, s1 = upper or
 * left site).  e_bonds (host, optional) = [Lx][Ly][2] horizontal, vertical
 * bond energies of each site. */
ctm_status ctm_energy(ctm_ctx* ctx, const double* h_host, double* e_site, double* e_bonds);

/* As ctm_energy with a different Hamiltonian on the horizontal bonds
 * (h_host, s1 = left site) and on the vertical bonds (hv_host, s1 = upper
 * site), same layout.  This is what a coarse-grained lattice needs, e.g. the
 * honeycomb lattice with two sites per tensor (p = 4), where the two bond
 * directions couple different sub-sites and an on-site term can be shared
 * out over the four bonds of a site. */
ctm_status ctm_energy_hv(ctm_ctx* ctx, const double* h_host, const double* hv_host, double* e_site, double* e_bonds);

/* Sec. III (the gradient of the variational energy by reverse-mode
 * differentiation through the CTMRG, at the cost of the CTMRG itself):
 * E(A) = energy after exactly n_sweeps sweeps from the start environment, and
 * dE/dA (device, FP64, layout of A, written by the call; the caller owns it)
 * by reverse mode with the hand-written adjoints; the environment is
 * checkpointed every ckpt_every sweeps and the sweeps of each block are
 * recomputed in the backward pass.  The current environment is left at the
 * state after the n_sweeps sweeps (also when n_sweeps is not a multiple of
 * ckpt_every).  CTM_EINVAL for n_sweeps < 0, ckpt_every < 1, NULL pointers
 * or a workspace sized for fewer sweeps per block; CTM_ENUMERIC for a
 * non-finite energy. */
ctm_status ctm_energy_grad(ctm_ctx* ctx, const double* h_host, int n_sweeps, int ckpt_every, double* e_site,
                           double* dA_dev);
/* As ctm_energy_grad with separate horizontal (h_host) and vertical
 * (hv_host) bond Hamiltonians, as in ctm_energy_hv. */
ctm_status ctm_energy_grad_hv(ctm_ctx* ctx, const double* h_host, const double* hv_host, int n_sweeps,
                              int ckpt_every, double* e_site, double* dA_dev);

/* Current environment to / from a device FP64 buffer in the packed layout
 * (ctm_env_elems doubles).  Import also resets the start environment. */
size_t ctm_env_elems(const ctm_config* cfg);
ctm_status ctm_env_export(ctm_ctx* ctx, double* env_dev);
ctm_status ctm_env_import(ctm_ctx* ctx, const double* env_dev);

/* Counters of the last call: algorithmic GEMM flops issued and Jacobi sweeps. */
ctm_status ctm_last_stats(ctm_ctx* ctx, double* gemm_flops, double* svd_sweeps);

/* Diagnostics: the kernels behind the calls above, exposed for kernel-level
 * checks.  ctm_debug_gemm: C[M][N] = op(A) op(B), row-major, prec CTM_FP64
 * (double) or CTM_FP32 / CTM_BF16X3 / CTM_BF16X6 (float); transA: A stored K x M, transB: B
 * stored N x K.  work: NULL, or device scratch of ctm_debug_gemm_work_bytes
 * bytes; when that size is nonzero the product runs as the contractions of
 * the library run it: split over K (long K, few 64 x 64 output tiles), or,
 * for BF16X3 products of 2^31 multiply-adds or more with both output
 * dimensions >= 1024, on operands split once into k-contiguous bf16 planes
 * (128 x 128 tiles, K sliced when the tiles are few).
 * ctm_debug_svd: batch n x n FP64 matrices M (n <= 4096, row-major, consecutive) ->
 * U S V^T, S descending; work = ctm_debug_svd_work_bytes bytes of device
 * memory; *sweeps in: sweep cap (<= 0: 60), out: sweeps run.  Both
 * synchronise the stream. */
size_t ctm_debug_gemm_work_bytes(int prec, int M, int N, int K);
ctm_status ctm_debug_gemm(int prec, int transA, int transB, int M, int N, int K, const void* A, const void* B,
                          void* C, void* work, void* hip_stream);
size_t ctm_debug_svd_work_bytes(int n, int batch);
/* ctm_debug_qr: Householder QR of batch tall matrices X (m x k, k <= m <=
 * 8192) given transposed, Xt = X^T (k x m row-major, consecutive; overwritten
 * by the reflectors and R).  R (k x k row-major, zero below the diagonal) and
 * Qt = Q^T (k x m) receive the thin factors (either may be NULL); work =
 * ctm_debug_qr_work_bytes bytes of device memory.  Synchronises the stream. */
size_t ctm_debug_qr_work_bytes(int m, int k, int batch);
ctm_status ctm_debug_qr(int m, int k, int batch, double* Xt, double* R, double* Qt, void* work, void* hip_stream);
ctm_status ctm_debug_svd(int n, int batch, const double* M, double* U, double* S, double* V, void* work,
                         int* sweeps, void* hip_stream);

/* Kernel timing (diagnostics): with on = k >= 1, every k-th launch of each
 * timed kernel class made by this context carries a start and a stop event
 * recorded by the runtime at the start and the end of that kernel on the
 * context's stream (k = 1: every launch; larger k keeps the events' own host
 * cost out of the run); on = 0 disables, on < 0 is CTM_EINVAL.  After each
 * call the sampled elapsed times are added up per class.  Enabling (or
 * disabling) resets the totals.  Classes: 0 GEMM FP64, 1 GEMM FP32, 2 GEMM
 * BF16x3, 3 Jacobi pair kernels (Gram matrix, test and 32 x 32
 * eigensolve of every block pair), 4 unused, 5 Jacobi rotations of G and V,
 * 6 GEMM BF16x6.  *ms = kernel time (the mean of the
 * sampled launches times the number of launches), *launches = number of
 * launches, *flops and *bytes = algorithmic work and memory traffic of those
 * launches (GEMM: 2 M N K flops and the operands read and written once;
 * pair kernels: the pairs' columns read once and the rotations written;
 * rotation: the rotated columns of G and V read and
 * written once, counted on the device for the pairs that were rotated). */
ctm_status ctm_kernel_timing_enable(ctm_ctx* ctx, int on);
ctm_status ctm_kernel_timing(ctm_ctx* ctx, int kernel_class, double* ms, double* launches, double* flops,
                             double* bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * ctm_init, but the workspace is the library's own static device array of
 * CTM_STATIC_SCRATCH_BYTES, one per GPU, held from the library's first use on
 * that GPU until the process ends.  The caller still passes A (device) and
 * keeps ownership of it and of every output buffer; nothing is allocated.
 * The array serves one context per device at a time: a second call on a
 * device whose array belongs to a live context (until its ctm_destroy) is
 * CTM_EINVAL, as is a configuration whose ctm_workspace_size (forward calls)
 * exceeds the array; calls with a larger transient need (e.g. ctm_energy_grad
 * over long checkpoint blocks) fail with CTM_EINVAL as with too small a
 * workspace.  The array keeps the last context's contents: nothing in it is
 * assumed to start at zero.  The device is the one current at the call;
 * CTM_EDEVICE if it cannot be queried. */
#define CTM_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
ctm_status ctm_init_static(const ctm_config* cfg, const double* A_dev, const double* boundary_vec_host,
                           void* hip_stream, ctm_ctx** out);

void ctm_destroy(ctm_ctx* ctx);
const char* ctm_strerror(ctm_status s);

#ifdef __cplusplus
}
#endif

#endif /* SPLITCTM_H */
