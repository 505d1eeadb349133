/*
 * ddgmres.h -- C ABI of the MI355X (gfx950) data-driven GMRES library.
 *
 * Solves the 2D frequency-domain Maxwell equation for E_z (Sec. 2, Eq. 1),
 *     [curl curl - omega^2 eps(x)/c^2] E = -i omega mu0 J,
 * discretised on the Yee grid with stretched-coordinate PML backed by
 * periodic boundaries, A f = b, by GMRES (Eq. 2) whose Krylov space is
 * augmented with a predicted subspace span(v_1..v_N) (Eqs. 3-5; the
 * supplement's update rule: QR of A V, projected Arnoldi, block least squares).
 *
 * Conventions
 *   - Units c = mu0 = eps0 = 1, lengths in micrometres, omega = 2 pi / lambda,
 *     time dependence exp(+i omega t); PML stretch s = 1 - i sigma/omega.
 *   - Grids are row-major with x fastest: flat index = iy*nx + ix, D = nx*ny.
 *   - Complex vectors are interleaved (re, im): DD_C64 = 2 x float (8 B),
 *     DD_C128 = 2 x double (16 B), the memory layout of torch.complex64/128.
 *   - Pointers are DEVICE pointers unless marked (host).
 *   - Work is ordered on the given stream; a call returns once its work is
 *     enqueued unless stated otherwise.  Calls that report results on the
 *     host (dd_solver_solve, gmres_solve*) synchronise the stream.
 *   - No C++ exception crosses this boundary.  Every non-OK status leaves a
 *     message for dd_last_error() (per thread).
 */
#ifndef DDGMRES_H
#define DDGMRES_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DD_OK = 0,
  DD_NOT_CONVERGED = 1, /* iteration budget spent; x holds the last iterate  */
  DD_EINVAL = -1,       /* invalid argument (sizes, omega, dx, pml, tol ...)   */
  DD_ENOMEM = -2,       /* device or host allocation failed                    */
  DD_EHIP = -3,         /* a HIP runtime call failed                           */
  DD_ENONFINITE = -4    /* non-finite permittivity or right-hand side          */
} dd_status;

typedef enum { DD_C64 = 0, DD_C128 = 1 } dd_prec;

/* Diagonal preconditioners of the comparison in the paper's supplement
 * (Table 1, data-free preconditioners).  The solver iterates on
 * A' = P_L A P_R, b' = P_L b, and recovers x = P_R x'.
 *   DD_PRECOND_JACOBI: P_L = diag(A)^{-1}, P_R = I.
 *   DD_PRECOND_PML:    P_L = S^{1/2}, P_R = S^{-1/2}, where
 *                      S = diag(s_x(i) s_y(j)) holds the PML stretch factors.
 *                      S A is complex symmetric, so P_L A P_R is complex
 *                      symmetric with the spectrum of A.  This is the reading
 *                      of the grid-spacing preconditioner of the paper's
 *                      Ref. 17. */
typedef enum { DD_PRECOND_NONE = 0, DD_PRECOND_JACOBI = 1, DD_PRECOND_PML = 2 } dd_precond;

/* PML description (host struct).  The profile is sigma(d) = sigma_max (d/n)^m
 * with sigma_max = -(m+1) ln_R / (2 n dx), d = depth in cells (integer and
 * half-integer positions, clamped to n).  The paper names PML without
 * parameters (Sec. 2); grade_m = 3, ln_R = -16 are the defaults used here.
 * npml_x / npml_y = 0 disables the layer on that axis. */
typedef struct {
  int npml_x, npml_y;
  int grade_m;
  double ln_R;
} dd_pml;

typedef struct fdfd_op fdfd_op;
typedef struct dd_solver dd_solver;
typedef struct dd_cnn dd_cnn;
typedef struct dd_predictor dd_predictor;

/* ------------------------------------------------------------------------
 * FDFD operator (Sec. 2, Eq. 1 and the paragraph after it)
 * ------------------------------------------------------------------------ */

/* Create the operator A = -(Dxb Dxf + Dyb Dyf) - omega^2 diag(eps).
 *   eps   (host) [ny][nx] relative permittivity, copied; may be freed on return.
 *   nx, ny >= 3; omega > 0; dx > 0; 2*npml < n on each axis.
 *   stream: the copies of eps and of the stencil coefficients (computed in
 *   FP64 on the host) are enqueued on it; the call synchronises it before
 *   returning.
 * Errors: DD_EINVAL for bad sizes/parameters, DD_ENONFINITE for non-finite
 * eps, DD_ENOMEM / DD_EHIP on allocation or copy failure (op left NULL).
 * The operator owns its device buffers until fdfd_op_destroy. */
dd_status fdfd_op_create(const float* eps, int nx, int ny, double omega, double dx,
                         const dd_pml* pml, hipStream_t stream, fdfd_op** op);

/* y = A x for one vector of D elements in precision p (x and y must not
 * alias).  Enqueued on stream. */
dd_status fdfd_op_apply(const fdfd_op* op, const void* x, void* y, dd_prec p,
                        hipStream_t stream);

/* Grid size of an operator (host out-params); returns D or -1 on NULL. */
int fdfd_op_dims(const fdfd_op* op, int* nx, int* ny);

void fdfd_op_destroy(fdfd_op* op);

/* ------------------------------------------------------------------------
 * Data-driven GMRES solver (Sec. 2, Eqs. 2-5; supplement Sec. 1)
 * ------------------------------------------------------------------------
 * A solver object holds the workspace for a batch of nb problems (one
 * operator each, sizes may differ) that are iterated in lockstep: every
 * kernel launch advances all unfinished problems by one step.
 *
 * Per cycle (restart length m): r = b - A x in FP64; c0 = C^H r and the
 * projected start r~ = r - C c0 (C from the thin QR A V = C R); Arnoldi on
 * P A (P = I - C C^H) with classical Gram-Schmidt run cgs_passes times over
 * [C, Q]; the Hessenberg matrix, its Givens rotations and the residual
 * estimate are kept in FP64; when the estimate drops to tol*||b|| (or after
 * m steps) the block least-squares problem of the supplement is solved
 * (x_aug = c0 - B y, B = C^H A Q) and x += V R^{-1} x_aug + Q y in FP64.
 * A new cycle starts from the recomputed FP64 residual; the solve has
 * converged when ||b - A x|| / ||b|| <= tol.
 */
typedef struct {
  dd_prec inner;        /* precision of matvecs and Gram-Schmidt (DD_C64 default) */
  int cgs_passes;       /* 1 = classical Gram-Schmidt, 2 = CGS2 (default)          */
  int restart;          /* m >= 1 (default 100)                                     */
  int kmax;             /* largest number of augmenting vectors, 0..64 (default 0) */
  int elems_per_thread; /* field elements per thread: 1, 2, 4, 8; 0 (default) = 8 */
                        /* for batches of >= 512 chunks of 2048 elements, else 2; */
                        /* -1 = the autotuner's choice (dd_solver_autotune, run   */
                        /* once per process for each set of grid sizes and        */
                        /* options, then remembered)                              */
  int hist_cap;         /* residual-history entries kept per problem (default 0)   */
  int check_every;      /* steps between host checks for an early cycle end (4)    */
  int select_reorth;    /* with cgs_passes = 2: run the second pass only in steps  */
                        /* where the first removed more than half of ||A q||^2    */
                        /* (Kahan-Parlett "twice is enough" test); default 1      */
  int use_graph;        /* 1 = replay groups of check_every Arnoldi steps as HIP   */
                        /* graphs (captured on first use; default 0)              */
  int precond;          /* dd_precond (default DD_PRECOND_NONE).  With a left     */
                        /* preconditioner the Givens estimate, the history and    */
                        /* rel_res_est are those of P_L r / ||P_L b||; convergence */
                        /* is still decided by the FP64 ||b - A x|| / ||b||        */
  void* workspace;      /* caller-owned device workspace (NULL: the solver         */
                        /* allocates its own); 256-byte aligned, at least the     */
                        /* size dd_solver_workspace_bytes reports for the same    */
                        /* operators and options; borrowed until destroy          */
  size_t workspace_bytes;
  int fused;            /* 1 = one sweep per Arnoldi step where it applies        */
                        /* (cgs_passes = 1, kmax + restart + 1 <= 128): the       */
                        /* update of step j, the matvec and the dots of step j+1  */
                        /* read each basis vector from memory once (30-column     */
                        /* strips walked down bands of rows); faster for one      */
                        /* problem alone, slower for batches; 0 (default) = two   */
                        /* sweeps per step                                        */
} dd_solver_opts;

/* Per-problem result (host struct). */
typedef struct {
  int status;          /* DD_OK or DD_NOT_CONVERGED                              */
  int iters;           /* Arnoldi steps (the paper's "iterations")               */
  int matvecs;         /* every application of A: setup k + steps + residuals   */
  int restarts;        /* cycles started                                         */
  int k_used;          /* augmenting columns kept after rank checks             */
  int fallback_plain;  /* 1 if a subspace was given but no column was usable     */
  int reorth_steps;    /* Arnoldi steps that took the second Gram-Schmidt pass   */
  double rel_res_true; /* ||b - A x|| / ||b|| recomputed in FP64 at the end      */
  double rel_res_est;  /* last Givens residual estimate / ||b||                  */
} dd_info;

void dd_solver_opts_default(dd_solver_opts* o);

/* Device bytes of the workspace a solver for these operators and options
 * needs (*bytes, host out): every vector, the FP64 small state and the
 * partial-sum rows, carved from one block.  No device memory is touched. */
dd_status dd_solver_workspace_bytes(const fdfd_op* const* ops, int nb,
                                    const dd_solver_opts* opts, size_t* bytes);

/* The same for one problem with k augmenting vectors, restart m and inner
 * precision (other options at their defaults), as gmres_solve uses it;
 * 0 on invalid arguments. */
size_t gmres_workspace_bytes(const fdfd_op* op, int k, int restart, dd_prec inner);

/* Allocate the workspace for nb problems, or take it from opts->workspace
 * (then the solver allocates no device memory; the caller keeps ownership
 * and must keep it alive until dd_solver_destroy).  ops (host array of nb
 * operator handles) are borrowed until destroy or the next dd_solver_bind.
 * Errors: DD_EINVAL (nb < 1, restart < 1, kmax outside 0..64, bad
 * elems_per_thread), DD_ENOMEM / DD_EHIP. */
dd_status dd_solver_create(const fdfd_op* const* ops, int nb, const dd_solver_opts* opts,
                           dd_solver** out);

/* Replace the operators of an existing solver by operators of the same grid
 * sizes (slot by slot).  Clears any subspace.  DD_EINVAL on a size mismatch. */
dd_status dd_solver_bind(dd_solver* s, const fdfd_op* const* ops);

/* Augmentation setup (supplement: QR of A V, storage of R^{-1}).
 * U (host array of nb device pointers, entries may be NULL) points to
 * [k[p]][D_p] vectors in the solver's inner precision; k (host) per problem,
 * 0 <= k[p] <= kmax; U == NULL or k == NULL clears all subspaces.
 * Computes W = A U, then C = W R^{-1} by Cholesky QR applied twice with the
 * Gram matrices accumulated in FP64; a column whose Cholesky pivot falls
 * below 1e-6 of the largest is dropped (k_used reports the rest), columns
 * with non-finite entries are dropped.  The vectors are copied; U may be
 * reused once the stream has passed this call. */
dd_status dd_solver_set_subspace(dd_solver* s, const void* const* U, const int* k,
                                 hipStream_t stream);

/* Solve all nb problems.  b[p]: [D_p] c128 right-hand side; x0 (host array,
 * may be NULL, entries may be NULL = zero start): [D_p] c128 initial guess;
 * x[p]: [D_p] c128 output (may alias x0[p]).  tol >= 0, maxit >= 0 (Arnoldi
 * steps per problem).  info (host, may be NULL) receives nb records.
 * Synchronises the stream.  Returns DD_OK if every problem converged,
 * DD_NOT_CONVERGED otherwise (x then holds the last iterate), DD_ENONFINITE
 * if a right-hand side is not finite, DD_EINVAL / DD_EHIP on errors.
 * ||b|| = 0 gives x = 0, DD_OK, rel_res_true = 0. */
dd_status dd_solver_solve(dd_solver* s, const void* const* b, const void* const* x0,
                          double tol, int maxit, void* const* x, dd_info* info,
                          hipStream_t stream);

/* Copy problem p's residual history (Givens estimate / ||b|| after each
 * Arnoldi step of the last solve, up to hist_cap entries) to host out[cap];
 * *n receives the number of entries written. */
dd_status dd_solver_history(const dd_solver* s, int p, double* out, int cap, int* n);

/* Subspace recycling along a sequence of related systems (Sec. 1: Krylov
 * information from earlier solves of related systems carried into the next
 * solve; supplement Sec. 1: GCROT keeps a few correction directions from
 * one cycle to the next).  After dd_solver_solve, for every problem p: the
 * search space of its last cycle is S = [U, Q_n] (U = V R^{-1}, the
 * augmenting directions with A U = C; Q_n the cycle's Arnoldi vectors), and
 * A S = W G with W = [C, Q_{n+1}] orthonormal and G = [[I, B], [0, H]] (the
 * matrix of eq:final_lsq).  The harmonic Ritz pairs (theta, y = S u), with
 * A y - theta y orthogonal to A S, solve G^H G u = theta G^H (W^H S) u; the
 * kout[p] = min(kr, dim S) of smallest |theta| are written to Y[p] as
 * [kout[p]][D] row-major complex vectors in the solver's inner precision
 * (complex64 or complex128), each scaled so that ||A y|| = 1, for
 * dd_solver_set_subspace of the next system (only their span matters).
 *   Y:     nb device pointers, caller-owned, room for kr vectors each;
 *          left untouched where kout[p] = 0 (no cycle ran and no subspace).
 *   kout:  host [nb], the number of vectors written per problem.
 *   theta: optional host [nb][kr] complex doubles (re, im interleaved): the
 *          harmonic Ritz values, infinite for a zero eigenvalue; zero past
 *          kout[p].
 * The device forms W^H V over the field and Y = S Z; the small eigenproblem
 * (Householder least squares, Hessenberg QR to Schur form, reordering) runs
 * on the host in FP64, one host thread per problem up to 16.  Allocates
 * device scratch of about 16 (kmax + restart + 1) kmax + 16 kr (kmax +
 * restart) bytes per problem and frees it; synchronises the stream.
 * Works on both Arnoldi paths (two sweeps, or one sweep with every Krylov
 * vector stored unnormalised, which the dots and the combination rescale).
 * Errors: DD_EINVAL (kr outside 1..64, NULL arguments, a preconditioner in
 * use, or no solve since the last set_subspace, bind or solve error),
 * DD_ENONFINITE (a rank-deficient small problem or no Schur convergence),
 * DD_ENOMEM / DD_EHIP. */
dd_status dd_solver_recycle(dd_solver* s, int kr, void* const* Y, int* kout, double* theta,
                            hipStream_t stream);

/* Host only: the small eigenproblem of dd_solver_recycle on its own.  G and
 * M = W^H S are nw x ns complex matrices (row-major, re/im interleaved) with
 * A S = W G, W orthonormal, G of full column rank, ns <= nw.  Writes to Z
 * (ns x kr, row-major complex) an orthonormal basis of the invariant
 * subspace of G^+ M for its kr eigenvalues of largest magnitude (the
 * harmonic Ritz values of smallest magnitude), columns scaled so that
 * ||G z|| = 1, and to theta (kr complex) those harmonic Ritz values in
 * increasing magnitude.  Errors: DD_EINVAL (sizes), DD_ENONFINITE (rank
 * deficiency, no convergence). */
dd_status dd_harmonic_ritz_host(int ns, int nw, const double* G, const double* M, int kr,
                                double* Z, double* theta);

/* Test introspection: copy an internal array of problem p to host memory.
 * what: 0 = C [k][D] (inner precision), 1 = Q [m+1][D] (after a full cycle the
 * last slot holds the new Arnoldi vector before normalisation, of norm
 * H[m-1][m]), 2 = H [m][m+1]
 * (FP64 complex, column-major, as built before rotation), 3 = B = C^H A Q
 * [m][k] (FP64 complex), 4 = R^{-1} [k][k] (FP64 complex, row-major).
 * bytes must match the array size exactly; synchronises the device. */
dd_status dd_solver_debug_copy(const dd_solver* s, int p, int what, void* host_out,
                               size_t bytes);

/* Live timing of the streaming sweeps of an Arnoldi step, recorded with HIP
 * events on the solve stream around every launch while enabled:
 * [0] stencil matvec + first Gram-Schmidt dots (with the fused sweep: the
 * first matvec of each cycle), [1] second Gram-Schmidt pass (update + dots),
 * [2] final update + norm, [3] fused sweep.  bytes[] are the algorithmic
 * bytes those launches had to move (inner precision ib bytes per complex, eb
 * per permittivity value, n = basis length of the step):
 * [0] (2 ib + eb) D + ib D n, [1] ib D (2n + 2), [2] ib D (n + 2),
 * [3] ib D (n + 3) + eb D (read the n basis vectors and A q~_j, write q~_{j+1}
 * and A q~_{j+1}, read eps). */
typedef struct {
  double ms[4];
  long long launches[4];
  double bytes[4];
} dd_kernel_stats;

/* Tile-shape autotuner: times one restart cycle of Arnoldi steps on ops for each
 * elements-per-thread value in {1, 2, 4, 8} (restart, precision and
 * Gram-Schmidt options from opts, right-hand sides of ones) and writes the
 * fastest to *best; ms_per_step (host, may be NULL) receives the 4 timings.
 * Allocates and frees its own workspace; synchronises the device. */
dd_status dd_solver_autotune(const fdfd_op* const* ops, int nb, const dd_solver_opts* opts,
                             int* best, double* ms_per_step);

/* Enable (1) or disable (0) the timing (graph replay is off while timing);
 * enabling resets the statistics. */
dd_status dd_solver_profile(dd_solver* s, int enable);
/* Host copy of the accumulated statistics. */
dd_status dd_solver_kernel_stats(const dd_solver* s, dd_kernel_stats* out);

/* Field elements per thread the solver runs with (the tile width chosen by
 * the rule or the autotuner; 0 for a NULL solver). */
int dd_solver_elems_per_thread(const dd_solver* s);

/* Device bytes of the solver workspace (its own or the caller's). */
size_t dd_solver_device_bytes(const dd_solver* s);

void dd_solver_destroy(dd_solver* s);

/* One-call convenience wrappers: create a solver, set the subspace, solve,
 * destroy.  U: [k][D] in the inner precision or NULL; opts may be NULL
 * (defaults).  Same status rules as dd_solver_solve. */
dd_status gmres_solve(const fdfd_op* op, const void* b, const void* x0, const void* U, int k,
                      double tol, int restart, int maxit, const dd_solver_opts* opts, void* x,
                      dd_info* info, hipStream_t stream);
dd_status gmres_solve_batched(const fdfd_op* const* ops, int nb, const void* const* b,
                              const void* const* x0, const void* const* U, const int* k,
                              double tol, int restart, int maxit, const dd_solver_opts* opts,
                              void* const* x, dd_info* info, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Principal-component basis (Sec. 3, PCA paragraph)
 * ------------------------------------------------------------------------
 * Leading left singular vectors of the uncentred snapshot matrix S whose M
 * columns are solution fields (an "incomplete SVD").  Computed as the FP64
 * Gram matrix G = S^H S on the device, its leading eigenpairs on the host
 * (FP64 Lanczos with full reorthogonalisation; the small tridiagonal matrix
 * is diagonalised by Jacobi rotations every ten steps to test convergence),
 * U = S W diag(1/sigma) on the device, then re-orthonormalised by Cholesky
 * QR.
 *   S:  [M][D] c64 snapshots (device), M >= k >= 1.
 *   U:  [k][D] c64 output basis (device).
 *   sigma (host, may be NULL): k singular values, descending.
 * Synchronises the stream. */
dd_status pca_build(const void* S, int M, int D, int k, void* U, double* sigma,
                    hipStream_t stream);

/* Training targets of the convolutional predictor from one trajectory of
 * solution fields F [S][D] c64 (device): for step s, U_loc = the leading k
 * left singular vectors of the unit-normalised fields of steps
 * s-window .. s+window, and target j = u_j (u_j^H f_s) with f_s normalised
 * (ordered by singular value, independent of the singular vectors' phases).
 * T: [S][k][D] c64 output (device); targets beyond the window's rank are 0.
 * Synchronises the stream. */
dd_status local_pca_targets(const void* F, int S, int D, int window, int k, void* T,
                            hipStream_t stream);

/* ------------------------------------------------------------------------
 * Projection loss of a subspace (Sec. 3, eq:proj_loss), batched evaluation
 * ------------------------------------------------------------------------
 * l = 1 - ||Q^H f||^2 / ||f||^2 with Q an orthonormal basis of span(V).
 * V: [nb][k][D] c64, f: [nb][D] c128 (device); out (host) [nb].
 * Synchronises the stream. */
dd_status proj_loss_batched(const void* V, const void* f, int nb, int k, int D, double* out,
                            hipStream_t stream);

/* ------------------------------------------------------------------------
 * Residual loss of a subspace (Sec. 3, eq:res_loss), batched evaluation
 * ------------------------------------------------------------------------
 * l_p = min_c ||A_p V_p c - b_p||^2 / ||b_p||^2, computed as
 * 1 - b^H P_W b / ||b||^2 with W = A V.  The FP64 Gram matrix of [W b] is
 * formed on the device; the k x k Cholesky solve runs on the host.  A
 * rank-deficient W gets a tiny ridge.
 *   ops[p]:  operator of problem p.
 *   b[p]:    [D] c128 (device).
 *   V[p]:    [k][D] c64 (device).
 *   out:     [nb] (host), clamped to [0, 1].
 * Problems may have different grids.  Synchronises the stream. */
dd_status res_loss_batched(const fdfd_op* const* ops, const void* const* b, const void* const* V,
                           int nb, int k, double* out, hipStream_t stream);

/* Residual loss and its gradient with respect to the subspace (Sec. 3,
 * eq:res_loss), the quantity the residual-loss training feeds into the
 * network's backward pass.  With c the least-squares coefficients and
 * r = b - A V c, the conjugate (Wirtinger) gradient is
 *     G = dl / d conj(V) = -(A^H r) c^H / ||b||^2,
 * so dl / d Re V = 2 Re G and dl / d Im V = 2 Im G.
 *   ops, b, V, nb, k, out: as res_loss_batched.
 *   G[p]: [k][D] c64 output (device, host array of nb pointers); column j is
 *         -(A^H r) conj(c_j) / ||b||^2.
 * Matvecs and r in complex64, the Gram matrix FP64, c FP64 on the host.
 * Scratch is allocated and freed inside the call.  Synchronises the stream. */
dd_status res_loss_grad_batched(const fdfd_op* const* ops, const void* const* b,
                                const void* const* V, int nb, int k, double* out,
                                void* const* G, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Effective-index field (Sec. 3: the CNN's second input)
 * ------------------------------------------------------------------------
 * The paper gives its CNN an effective-index simulation of the field: a
 * cheap approximation obtained from 1D solves of Maxwell's equations.  The
 * separable reading computed here has three steps, for each problem p
 * (operator ops[p], right-hand side b[p]):
 *   1. phi_ix = fundamental mode (lowest eigenpair mu_ix, unit norm,
 *      positive) of the column operator
 *      -(second difference in y)/dx^2 - omega^2 eps(ix, .), with zero field
 *      outside the column;
 *   2. a solves the 1D equation along x.  It has the operator's stretched
 *      x-differences (PML, periodic wrap) and mu_ix in place of
 *      -omega^2 eps.  The source is j_ix = phi_ix^T b[:, ix];
 *   3. F[iy][ix] = a_ix phi_ix(iy).
 * All arithmetic is FP64.
 *   b[p]: [D] c128 (device).
 *   F[p]: [D] c64 output (device).
 * Problems may have different grids.  Scratch memory is allocated and freed
 * inside the call.  Synchronises the stream. */
dd_status eim_field(const fdfd_op* const* ops, int nb, const void* const* b, void* const* F,
                    hipStream_t stream);

/* eim_field without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, kernels and results as eim_field; its scratch
 * is a fixed device array of DD_EIM_NOALLOC_BYTES held by the library on
 * every GPU it runs on until the process ends (resolved once per device on
 * the first call there).  A batch needs 16 B per cell plus 120 B per grid
 * column plus 72 B per problem: 1.86 MB for one 480 x 240 grid, so up to 17
 * such problems per call.  A larger batch returns DD_EINVAL with a message
 * and runs nothing.  Every call on one GPU uses the same array: calls that
 * overlap on one GPU (other threads or streams) race and must be serialised
 * by the caller.  Synchronises the stream. */
#define DD_EIM_NOALLOC_BYTES 33554432
dd_status eim_field_noalloc(const fdfd_op* const* ops, int nb, const void* const* b,
                            void* const* F, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Convolutional subspace predictor (Sec. 3, CNN paragraph; Methods)
 * ------------------------------------------------------------------------
 * Encoder-decoder of eight 3x3 convolutions on a [B][ny][nx] permittivity
 * image (the architecture figure of the paper is not available; the layer
 * list is fixed by dd_cnn_layer_info).  Activations are bf16 in NHWC
 * layout, products accumulate in FP32 on the matrix cores, master weights
 * and Adam moments are FP32.  The first layer (input planes to 32 channels)
 * and its weight gradient run in FP32 throughout.  The 2k output channels are read as k complex
 * fields (channel 2j = real part, 2j+1 = imaginary part of v_j).
 */

/* Create a network for input images of ny x nx (both multiples of 4), up to
 * max_batch images per call and k output fields.  in_channels selects the
 * input:
 *   - 1: the permittivity alone;
 *   - 3: the permittivity plus the real and imaginary parts of the
 *     effective-index field (eim_field).  The field is scaled to unit RMS per
 *     pixel, per image.  The paper's CNN takes both inputs.
 * Weights are initialised from seed (He-uniform, host RNG, documented in the
 * source). */
dd_status dd_cnn_create(int nx, int ny, int max_batch, int k, int in_channels,
                        unsigned long long seed, dd_cnn** out);
void dd_cnn_destroy(dd_cnn* net);

/* Number of layers and, per layer (host out-params, may be NULL): input
 * channels, output channels, stride (1 or 2), upsample-before (0/1), relu (0/1). */
int dd_cnn_layer_info(const dd_cnn* net, int layer, int* cin, int* cout, int* stride,
                      int* upsample, int* relu);

/* Number of FP32 parameters (weights + biases) and host copies in / out in the
 * layout [layer][cout][cin][3][3] then [layer][cout] biases, layer by layer. */
size_t dd_cnn_num_params(const dd_cnn* net);
dd_status dd_cnn_get_params(const dd_cnn* net, float* host_out, size_t count);
dd_status dd_cnn_set_params(dd_cnn* net, const float* host_in, size_t count);

/* Forward pass of a one-input-channel network.
 *   eps: [B][ny][nx] float32 permittivity (device).  The input is normalised
 *        as (eps - 2.085) / (12.25 - 2.085).
 *   U:   [B][k][ny*nx] c64 output fields (device).
 *   B <= max_batch. */
dd_status dd_cnn_predict(dd_cnn* net, const float* eps, int B, void* U, hipStream_t stream);

/* Forward pass of a three-input-channel network.
 *   eim: [B][ny*nx] c64 effective-index fields (device, from eim_field).
 * Otherwise as dd_cnn_predict. */
dd_status dd_cnn_predict_eim(dd_cnn* net, const float* eps, const void* eim, int B, void* U,
                             hipStream_t stream);

/* Grid, output fields, input planes and batch capacity of a network (host
 * out-params, each may be NULL). */
dd_status dd_cnn_dims(const dd_cnn* net, int* nx, int* ny, int* k, int* in_channels,
                      int* max_batch);

/* Save a network to a predictor file: its configuration, the FP32 master
 * parameters and the Adam state (first and second moments, step count), so
 * that training resumes exactly where it stopped.  Synchronises the device. */
dd_status dd_cnn_save(const dd_cnn* net, const char* path /* (host) */);

/* Recreate a network saved by dd_cnn_save, for batches of up to max_batch
 * images.  DD_EINVAL (message set) if the file is missing, malformed,
 * truncated or holds a PCA basis. */
dd_status dd_cnn_load(const char* path /* (host) */, int max_batch, dd_cnn** out);

/* One training step on a batch:
 *   1. forward pass;
 *   2. mean-squared error against target [B][k][ny*nx] c64 (device, same
 *      layout as U);
 *   3. backward pass;
 *   4. Adam update with learning rate lr, betas (b1, b2) and epsilon 1e-8.
 * eim must be [B][ny*nx] c64 for a three-channel network and NULL for a
 * one-channel one.  *loss (host, may be NULL) receives the batch loss.
 * Synchronises the stream. */
dd_status dd_cnn_train_step(dd_cnn* net, const float* eps, const void* eim, const void* target,
                            int B, float lr, float b1, float b2, float* loss,
                            hipStream_t stream);

/* Gradient of the batch loss w.r.t. all parameters, with no update.
 * host_grad receives count FP32 values (host) in the dd_cnn_get_params
 * layout.  Used for gradient checks.  eim is as in dd_cnn_train_step. */
dd_status dd_cnn_grad(dd_cnn* net, const float* eps, const void* eim, const void* target, int B,
                      float* loss, float* host_grad, size_t count, hipStream_t stream);

/* Residual-loss training (Sec. 3, eq:res_loss; unsupervised).  The loss is
 * the batch mean of l_res of each image's predicted fields against its own
 * operator ops[p] (grid ny x nx) and right-hand side b[p] ([D] c128, device).
 * The gradient with respect to the fields is -(A^H r) c^H / ||b||^2 per
 * image, with c the least-squares coefficients and r = b - A V c.  It runs
 * through the network's backward pass, then an Adam update as in
 * dd_cnn_train_step.  eim is as in dd_cnn_train_step.  *loss (host, may be
 * NULL) receives the batch mean.  Synchronises the stream. */
dd_status dd_cnn_train_step_res(dd_cnn* net, const float* eps, const void* eim,
                                const fdfd_op* const* ops, const void* const* b, int B, float lr,
                                float b1, float b2, float* loss, hipStream_t stream);

/* Gradient of the batch residual loss with respect to all parameters, with
 * no update.  host_grad (host, count values) uses the dd_cnn_get_params
 * layout.  For gradient checks. */
dd_status dd_cnn_grad_res(dd_cnn* net, const float* eps, const void* eim,
                          const fdfd_op* const* ops, const void* const* b, int B, float* loss,
                          float* host_grad, size_t count, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Subspace predictor (Sec. 3: a model that maps the permittivity to the
 * vectors v_1..v_N augmenting GMRES; the PCA basis is the same for every
 * permittivity, the CNN specialises it)
 * ------------------------------------------------------------------------
 * A predictor file holds either a PCA basis (predictor_save_pca) or a CNN
 * with its Adam state (dd_cnn_save): a 48-byte header (magic "DDPRED01",
 * kind 1 = PCA / 2 = CNN, nx, ny, k, input planes, value count, Adam step)
 * followed by little-endian float32 data. */

/* Write the k basis vectors U [k][ny*nx] c64 (device) as a PCA predictor
 * file.  Synchronises the stream. */
dd_status predictor_save_pca(const char* path /* (host) */, const void* U, int k, int nx, int ny,
                             hipStream_t stream);

/* Load a predictor file for batches of up to max_batch problems (the CNN's
 * activation buffers are sized by it).  DD_EINVAL (message set) if the file
 * is missing, malformed or truncated; DD_ENOMEM / DD_EHIP on device errors.
 * The predictor owns its device memory until predictor_destroy. */
dd_status predictor_load(const char* path /* (host) */, int max_batch, dd_predictor** out);

/* Kind (1 PCA, 2 CNN), grid, k and input planes (0 for PCA) of a predictor
 * (host out-params, each may be NULL). */
dd_status predictor_info(const dd_predictor* p, int* kind, int* nx, int* ny, int* k,
                         int* in_channels);

/* U [B][k][ny*nx] c64 (device) = the predicted subspace of each of B
 * problems.
 *   PCA: the basis for every problem; eps may be NULL.
 *   CNN with one input plane: eps [B][ny][nx] float32 (device).
 *   CNN with three input planes: eps, plus ops (host array of B operators)
 *        and b (host array of B device [D] c128 right-hand sides) from which
 *        the effective-index field is computed (eim_field).
 * ops, when given, must be on the predictor's grid.  B <= max_batch for a
 * CNN.  The predictor's internal buffers are reused, so calls on one
 * predictor must not overlap.  Synchronises the stream. */
dd_status predict_subspace(dd_predictor* p, const fdfd_op* const* ops, const void* const* b,
                           const float* eps, int B, void* U, hipStream_t stream);

void predictor_destroy(dd_predictor* p);

/* Copy the bf16 activations of layer l's output (NHWC, as float32) to host.
 * layer = -1 gives the normalised input planes [B][in_channels][ny][nx].  The
 * last layer's FP32 output is read from where the last forward pass wrote it
 * (the caller's U for a prediction, which must still be allocated).
 * For tests. */
dd_status dd_cnn_debug_activation(const dd_cnn* net, int layer, int B, float* host_out,
                                  size_t count);

/* Last error message of this thread ("" if none). */
const char* dd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DDGMRES_H */
