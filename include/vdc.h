/*
 * vdc.h - C ABI of the MI355X (gfx950) solver for vibronic dynamics of
 * discrete states in the electron continuum.
 *
 * Method: Cosicova, Dvorak & Cizek, "Vibronic dynamics in electron continuum -
 * iterative solvers", arXiv:2307.13483.  The library builds the generalized
 * two-state, two-mode model of Sec. II.C and, for each job (incident energy
 * eps_i, initial vibrational state v_i, incoming partial wave mu_i), solves
 *     (E - H_ef(E)) Psi = Phi^{v_i mu_i},   E = eps_i + E_{v_i}     (Eqs. (2), (26))
 * by a Krylov method of Sec. III.A (restarted GMRES, or COCG with the
 * symmetrized bilinear form), right-preconditioned by a block-diagonal
 * section of A (Sec. III.B: its diagonal, column blocks or rows), in FP64 or
 * with FP32 inner solves inside an FP64 outer iteration, then projects the
 * T-matrix amplitudes (Eqs. (15), (24)) and cross sections (Eq. (16)).
 *
 * Conventions shared by every entry point
 *  - Energies in eV.  T is dimensionless; sigma is in bohr^2 with eps_i
 *    converted to hartree (1 hartree = 27.211386245988 eV) in 2 pi^3/eps_i.
 *  - Complex numbers are interleaved (re, im) pairs of double ("c16") or,
 *    where stated, float.
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller.  The library never
 *    keeps a caller pointer past the call.
 *  - Work is ordered on the caller's hipStream_t (passed as void*, NULL = the
 *    default stream).  Calls that return host results synchronise that stream.
 *  - Every function returns vdc_status; it never throws or aborts.  On error
 *    vdc_last_error() returns a thread-local message.  A job that fails to
 *    converge is not a call error: it is reported in its vdc_job_status.
 *  - Basis (Sec. II.D): compound index alpha = (d, n_g, n_u), d in {1,2},
 *    n_g < Ng, n_u < Nu; full vectors are laid out d-major, then n_g, with n_u
 *    fastest: index (d-1)*Ng*Nu + n_g*Nu + n_u, length N = 2*Ng*Nu.
 */
#ifndef VDC_H
#define VDC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VDC_OK = 0,
  VDC_ERR_INVALID_ARG = 1,   /* a size, pointer or parameter is out of range   */
  VDC_ERR_WORKSPACE = 2,     /* workspace smaller than vdc_workspace_size()     */
  VDC_ERR_HIP = 3,           /* a HIP runtime call failed                       */
  VDC_ERR_UNSUPPORTED = 4    /* a valid request the library does not implement */
} vdc_status;

typedef enum {
  VDC_CONVERGED = 0,         /* ||b - A x||_2 <= tol ||b||_2 (true residual)    */
  VDC_NOT_CONVERGED = 1,     /* max_iter reached first                          */
  VDC_BREAKDOWN = 2,         /* Krylov space exhausted without reaching tol     */
  VDC_NONFINITE = 3          /* a NaN/Inf appeared in the iteration             */
} vdc_job_status;

/* Parameters of the generalized model, Sec. II.C (Eqs. (18), (21)-(23)).
 *   H_0   = w_g (n_g + 1/2) + w_u (n_u + 1/2)
 *   U     = [[E1 + kappa1 q_g, lam q_u], [lam q_u, E1 + gap + kappa2 q_g]]
 *   V_eps = [[f_1^e (1 + lam1 q_g), f_1^o q_u], [f_2^e q_u, f_2^o (1 + lam2 q_g)]]
 *   2 pi (f_d^mu)^2 = Gamma_d^mu(eps) = A[d][mu] eps^(l[mu]+1/2) exp(-eps/B[d][mu]),
 *   f >= 0, Gamma = 0 for eps <= 0.  Index d: 0 -> state 1, 1 -> state 2;
 *   mu: 0 -> even (e), 1 -> odd (o).
 * The level shift F[f_d f_d'] (Eq. (19)) has the analytic imaginary part
 * -sqrt(Gamma_d Gamma_d')/2 and, as real part, the principal-value transform
 * of the piecewise-linear interpolant of sqrt(Gamma_d Gamma_d') on the nodes
 * x_k = (k sqrt(hilbert_xmax)/(hilbert_nodes-1))^2, k = 0..hilbert_nodes-1. */
typedef struct {
  double omega_g, omega_u;
  double kappa1, kappa2, lam;
  double lam1, lam2;
  double E1, gap;
  double A[2][2];            /* [d][mu], >= 0                                    */
  double B[2][2];            /* [d][mu], > 0                                     */
  int l[2];                  /* [mu], 0..4, the same for both states            */
  int Ng, Nu;                /* basis sizes, 1..1024 each                       */
  int hilbert_nodes;         /* 16..65536 (4096 in the reference workloads)     */
  double hilbert_xmax;       /* > 0 eV (40 in the reference workloads)          */
} vdc_model2d_desc;

typedef struct vdc_model* vdc_model_t;   /* opaque; owns a few KB of device data */

/* One right-hand side.  v_i = (vi_g, vi_u) must lie in the basis and
 * eps_i > 0 (an open entrance channel), else the call fails with
 * VDC_ERR_INVALID_ARG.  model indexes the models[] array of the call.      */
typedef struct {
  double eps_i;
  int vi_g, vi_u;
  int mu_i;                  /* 0 = e, 1 = o                                    */
  int model;
} vdc_job;

/* Right preconditioners (Sec. III.B), each a block-diagonal section of A:
 * JACOBI its diagonal; BLOCK the blocks of one n_u column and 8 consecutive
 * n_g (the paper's M^u cut into segments); ROWS one block per n_g holding
 * its whole n_u row with both states (the paper's M^g, 2 N_u x 2 N_u, of
 * which each symmetry block holds one half).  Blocks are factored once per
 * job by complex symmetric LDL^T (in FP64; with VDC_FP32_INNER the inner
 * solves apply a factor whose multipliers are stored in FP16 and 1/D in
 * FP32, exactly as stored, so it stays symmetric); a block with a vanishing
 * pivot, or whose multipliers leave the FP16 range in that mode, falls back
 * to its diagonal.  ROWS factors and applies each row serially (one thread
 * per row, N_g threads of a job): cheap per step, but its worth is the
 * iteration count, which it cuts most where lam q_u is the strong coupling.
 * The CO2-like model takes NONE, JACOBI or BLOCK (its own block choice). */
typedef enum {
  VDC_PREC_NONE = 0,
  VDC_PREC_JACOBI = 1,
  VDC_PREC_BLOCK = 2,
  VDC_PREC_ROWS = 3
} vdc_precond;
typedef enum {
  VDC_FP64 = 0,              /* the whole Krylov solve in complex FP64           */
  VDC_FP32_INNER = 1         /* FP64 outer iteration (true residual, Givens,
                                solution, amplitudes) around inner solves in
                                complex FP32 with FP32 accumulation: with
                                VDC_GMRES, FGMRES whose variable preconditioner
                                is FP32 GMRES; with VDC_COCG, FP64 iterative
                                refinement whose correction equations are
                                solved by FP32 COCG (see vdc_method)          */
} vdc_precision;

/* Krylov method of vdc_solve, the batch entry points, vdc_solve_adjoint and
 * vdc_co2_solve (Sec. III.A): restarted GMRES (with the precision above), or
 * COCG, conjugate gradients with the bilinear form <a|b>_S = sum a_i b_i for
 * the complex symmetric A, preconditioned as M^{-1} A M^{-T} with M M^T the
 * JACOBI, BLOCK or ROWS section (all symmetric).  Not for vdc_solve_plain.
 * COCG with VDC_FP32_INNER (not for the adjoint) is FP64 iterative refinement
 * whose correction equations are solved by COCG entirely in FP32 to the
 * relative residual inner_tol or inner_restart steps; iters then counts the
 * FP32 steps, outer_iters the refinements.  In FP64 restart is ignored, max_iter counts COCG steps, and the
 * true residual decides convergence (the iteration restarts from it when the
 * updated residual has converged but it has not).  A vanishing bilinear
 * form at a fresh start is VDC_BREAKDOWN. */
typedef enum { VDC_GMRES = 0, VDC_COCG = 1 } vdc_method;

typedef struct {
  int restart;               /* GMRES restart length m, 1..128                  */
  int max_iter;              /* total Arnoldi steps (inner steps for FP32)      */
  double tol;                /* relative true-residual target, > 0            */
  int precond;               /* vdc_precond                                     */
  int precision;             /* vdc_precision                                   */
  int inner_restart;         /* FP32_INNER: inner GMRES length (1..128), or
                                the inner COCG step limit (>= 1)             */
  double inner_tol;          /* FP32_INNER: inner relative tolerance            */
  int outer_restart;         /* FP32_INNER: outer FGMRES length (1..32)         */
  int tile_rows;             /* rows of n_g per LDS tile of the fused operator
                                pass; 0 = the largest that fits               */
  int method;                /* vdc_method (vdc_solve only; 0 = GMRES)         */
  int check_optical;         /* 1: compute vdc_job_info.optical_defect for every
                                two-state or term-list solve (one more pass
                                over the solution per job; the solve kernels
                                of that launch are the instantiations that
                                also write residual histories); 0: not
                                computed, optical_defect = -1                 */
} vdc_solve_opts;

/* Per-job results written to host memory by the solve calls. */
typedef struct {
  int status;                /* vdc_job_status                                  */
  int iters;                 /* Arnoldi steps taken (inner steps for FP32)      */
  int restarts;              /* GMRES cycles (outer steps for FP32)             */
  int outer_iters;           /* FP32_INNER: outer FGMRES steps, else 0          */
  double rel_res;            /* final ||b - A x|| / ||b||, FP64 true residual   */
  double alg_bytes;          /* HBM bytes the job's solve moves by the solver's
                                design (vector passes x element size; see the
                                byte model in the solver sources), excluding
                                the level-shift tables' construction           */
  int retried;               /* vdc_solve with VDC_FP32_INNER: 1 if the job did
                                not converge in the mixed-precision solve and
                                was solved again in FP64 (the other fields then
                                describe the FP64 solve), 2 if that re-solve
                                did not fit the workspace, else 0             */
  int reserved;
  double optical_defect;     /* |-Im T_ii - pi sum |T_f|^2| / |T_ii| of the
                                solution, the sum over every open final state
                                and partial wave of the basis: the truncated-
                                basis optical theorem, exact for the exact
                                solution (two-state and term-list solves with
                                opts.check_optical = 1; -1 where not computed:
                                check_optical = 0, the CO2-like model and the
                                adjoint)                                     */
} vdc_job_info;

/* Build a model (host call; allocates and fills its small device tables:
 * the transform's nodes and second differences of the interpolated widths). */
vdc_status vdc_model2d_create(const vdc_model2d_desc* desc, vdc_model_t* out);
vdc_status vdc_model_destroy(vdc_model_t model);

/* Bytes of device workspace that vdc_solve / vdc_solve_plain need for this job
 * list (for VDC_COCG: vdc_solve only).  Host call, no device work. */
vdc_status vdc_workspace_size(int n_models, const vdc_model_t* models,
                              const vdc_solve_opts* opts, int n_jobs, const vdc_job* jobs,
                              size_t* bytes);

/* Solve every job in ONE persistent kernel launch (after one launch that
 * builds the per-energy level-shift tables).  Each workgroup pops jobs,
 * longest-first, from a device queue and runs the whole restarted GMRES for
 * the job on chip, then projects the amplitudes.
 *   finals   host int[n_final][2]: (n_g, n_u) of each final state v_f
 *   T_out    device c16 [n_jobs][n_final][2]: T_{mu_f v_f <- mu_i v_i},
 *            mu_f = e, o; 0 for closed channels (eps_f <= 0)
 *   sigma_out device double [n_jobs][n_final]: this job's share of
 *            sigma_{v_f <- v_i}, 2 pi^3/eps_i sum_{mu_f} |T|^2; the cross
 *            section of Eq. (16) is the sum of the shares of the mu_i = e and
 *            mu_i = o jobs at the same (eps_i, v_i)
 *   psi_out  device c16 [n_jobs][N] or NULL: the solution Psi, full layout
 *   info     host vdc_job_info[n_jobs] or NULL
 * Requirements: workspace device, >= vdc_workspace_size() bytes, 256-byte
 * aligned.  Synchronises the stream before returning.
 * With VDC_FP32_INNER, every job that does not converge (FP32 stagnation, a
 * breakdown or a non-finite FP32 value) is solved again in FP64 with the same
 * method, preconditioner and limits, in the same workspace (with fewer
 * resident workgroups if needed), and marked in info[j].retried; its outputs
 * are then those of the FP64 solve.  The batch entry points do not retry
 * (they never synchronise): check vdc_batch_info. */
vdc_status vdc_solve(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                     int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                     void* workspace, size_t ws_bytes,
                     double* T_out, double* sigma_out, double* psi_out,
                     vdc_job_info* info, void* stream);

/* vdc_solve recording every job's convergence history (off in the other
 * calls): after each step, hist[j][k] (device double [n_jobs][hist_len],
 * row j = the caller's job j) receives the relative residual ||r||/||b|| that
 * the method tracks after step k + 1: GMRES the least-squares residual of
 * the Arnoldi step (Sec. III.A), FGMRES the outer one, COCG the updated
 * residual, FP32-inner COCG the inner residual times the outer residual norm
 * (one entry per FP32 step).  Entries past the job's last step, and steps
 * beyond hist_len, are not written.  No FP64 re-solve of FP32-inner jobs.
 * Otherwise as vdc_solve. */
vdc_status vdc_solve_history(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                             int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                             void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                             double* psi_out, vdc_job_info* info, double* hist, int hist_len,
                             void* stream);

/* vdc_solve for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid hipMalloc, code running while another stream
 * captures a HIP graph): the same plan, kernels and outputs as vdc_solve, with no
 * workspace argument.  The library keeps one static device array of
 * VDC_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU it runs on, held until the
 * process ends, and runs the call in it: with fewer resident workgroups when
 * the plan does not fit, and VDC_ERR_WORKSPACE (message names the bytes
 * needed) when even one workgroup's slot, the level-shift tables and the job
 * descriptors do not fit - e.g. a 120 x 120 batch over hundreds of energies;
 * use vdc_solve there.  No hipMalloc, hipFree or event is created; the
 * job descriptors are copied into the array with hipMemcpyAsync.  Kernel
 * times are not recorded (vdc_last_kernel_times keeps the previous call's).
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (each call initialises what it reads): calls that overlap on one
 * GPU, from several host threads or streams, race and must be serialised
 * by the caller.  Synchronises the stream before returning. */
#define VDC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vdc_status vdc_solve_noalloc(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                             int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                             double* T_out, double* sigma_out, double* psi_out,
                             vdc_job_info* info, void* stream);

/* The batched solve as a reusable launch (for host loops that repeat the same
 * jobs, and for capture into a HIP graph: the whole batch, tables included,
 * becomes one graph launch).
 * vdc_batch_create: the checks, plan and descriptor upload of vdc_solve, done
 *   once; the batch keeps the workspace and output pointers (caller-owned,
 *   they must stay allocated and unchanged until vdc_batch_destroy) and
 *   synchronises the stream before returning.  Same arguments as vdc_solve
 *   without info.  n_jobs >= 1.
 * vdc_batch_launch: enqueues the counter reset, the level-shift table
 *   kernels and the persistent solver on the stream: kernels only, no copy,
 *   memset, allocation or host synchronisation, so the call may be captured.
 * vdc_batch_capture: captures vdc_batch_launch on the stream (not the null
 *   stream) into a HIP graph owned by the batch and instantiates it
 *   (replacing an earlier one); vdc_batch_replay launches that graph.
 * vdc_batch_info: per-job results of the last completed launch or replay
 *   (synchronises the stream).
 * vdc_batch_kernel_times: milliseconds of the level-shift table kernels and
 *   of the solver kernel in the last vdc_batch_launch, from HIP events
 *   recorded on its stream (waits for them); replays are not timed.
 * Launches of one batch on several streams at once race on its workspace. */
typedef struct vdc_batch* vdc_batch_t;
vdc_status vdc_batch_create(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                            int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                            void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                            double* psi_out, void* stream, vdc_batch_t* out);
vdc_status vdc_batch_launch(vdc_batch_t batch, void* stream);
vdc_status vdc_batch_capture(vdc_batch_t batch, void* stream);
vdc_status vdc_batch_replay(vdc_batch_t batch, void* stream);
vdc_status vdc_batch_info(vdc_batch_t batch, vdc_job_info* info, void* stream);
vdc_status vdc_batch_kernel_times(vdc_batch_t batch, double* ms_tables, double* ms_solver);
vdc_status vdc_batch_destroy(vdc_batch_t batch);

/* The plain single-solve path: the same arithmetic, one job after another,
 * each GMRES step issued from the host as separate grid-wide kernels (matvec,
 * Gram-Schmidt projections, norm, Givens update) with one status read-back
 * per restart cycle.  FP64 only (opts->precision must be VDC_FP64).  Same
 * arguments and outputs as vdc_solve. */
vdc_status vdc_solve_plain(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                           int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                           void* workspace, size_t ws_bytes,
                           double* T_out, double* sigma_out, double* psi_out,
                           vdc_job_info* info, void* stream);

/* Gradient of a loss L(sigma) with respect to the 16 model parameters, by
 * the adjoint method: for each job, with its forward solution Psi and
 * amplitudes T (from vdc_solve with the same jobs and finals), one solve with
 * the same operator (A^T = A, Sec. III.A) of A zeta = sum_f W_f Phi^{v_f mu_f},
 * W_f = 2 (2 pi^3/eps_i) dL/dsigma_f conj(T_f), then
 *   dL/dp = Re[sum_f W_f (dPhi_f/dp)^T Psi + zeta^T dPhi_i/dp - zeta^T (dA/dp) Psi]
 * with the derivatives of Eqs. (18), (21)-(23), (25) (level shift
 * differentiated through the principal-value transform).  Parameter order:
 * omega_g, omega_u, kappa1, kappa2, lam, lam1, lam2, gap, A[0][0] (1e),
 * A[1][0] (2e), A[0][1] (1o), A[1][1] (2o), B in the same order.
 *   psi        device c16 [n_jobs][2*max(Ng*Nu)]: forward solutions (psi_out)
 *   T          device c16 [n_jobs][n_final][2]: forward amplitudes (T_out)
 *   dL_dsigma  device double [n_jobs][n_final]: dL/dsigma_{v_f <- v_i} at the
 *              job's (eps_i, v_i) (the same value for its mu_i = e and o jobs)
 *   grad_jobs  device double [n_jobs][16]: each job's contribution
 *   grad       host double[16] or NULL: sum over jobs (in job order)
 *   info       host vdc_job_info[n_jobs] or NULL: the adjoint solves
 * FP64 only; the transposed solves use opts->method (GMRES or COCG).
 * Workspace: vdc_adjoint_workspace_size().  Synchronises. */
vdc_status vdc_adjoint_workspace_size(int n_models, const vdc_model_t* models,
                                      const vdc_solve_opts* opts, int n_jobs,
                                      const vdc_job* jobs, size_t* bytes);
vdc_status vdc_solve_adjoint(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                             int n_jobs, const vdc_job* jobs, int n_final, const int* finals,
                             const double* psi, const double* T, const double* dL_dsigma,
                             void* workspace, size_t ws_bytes, double* grad_jobs, double* grad,
                             vdc_job_info* info, void* stream);

/* Level-shift tables (Eq. (19) with the widths of Eq. (22)): for n_eps
 * electron energies eps (device double[n_eps]) write the six complex values
 * F[f_1^e f_1^e], F[f_1^e f_2^e], F[f_2^e f_2^e], F[f_1^o f_1^o],
 * F[f_1^o f_2^o], F[f_2^o f_2^o] at each energy to out (device c16
 * [n_eps][6]).  Asynchronous on the stream. */
vdc_status vdc_level_shift(vdc_model_t model, int n_eps, const double* eps, double* out,
                           void* stream);

/* y = A x for the matrix A = E - H_ef(E) of Eq. (28) at total energy E, applied
 * to n_vec full-layout vectors x (device c16 [n_vec][N]) that each lie in one
 * symmetry block (parity[v] = 0: d=1 on even n_u and d=2 on odd n_u; 1: the
 * opposite; host int[n_vec]); components outside the block are ignored and
 * written as 0.  y: device c16 [n_vec][N].  workspace: device, >=
 * vdc_matvec_workspace_size() bytes.  Asynchronous on the stream. */
vdc_status vdc_matvec_workspace_size(vdc_model_t model, int n_vec, size_t* bytes);
vdc_status vdc_matvec(vdc_model_t model, double E, int n_vec, const int* parity,
                      const double* x, double* y, void* workspace, size_t ws_bytes,
                      void* stream);

/* Durations, in milliseconds, of the kernels of the last vdc_solve /
 * vdc_solve_plain call on this host thread, measured with HIP events recorded
 * on the call's stream: the level-shift table kernel and the solver (the
 * persistent kernel, or the whole sequence of plain-path kernels).  Host
 * pointers, either may be NULL. */
vdc_status vdc_last_kernel_times(double* ms_tables, double* ms_solver);

/* y = A x on vectors in the solvers' symmetry-block layout: n_vec vectors of
 * Ng*Nu complex values (device c16 [n_vec][Ng*Nu], n_g-major, n_u fastest),
 * vector v in block parity[v] (host int[n_vec]): at (n_g, n_u) the value is
 * the component of state 1 if n_u + parity is even, of state 2 otherwise.
 * One total energy E for all vectors; its level-shift tables are built first.
 * One wavefront per (vector, slab of n_g rows, strip of 60 n_u columns),
 * no LDS tiles or barriers.  x and y must not overlap.
 * Kernel times are reported by vdc_last_kernel_times (tables, operator).
 * Workspace: vdc_matvec_block_workspace_size().  Synchronises the stream. */
vdc_status vdc_matvec_block_workspace_size(vdc_model_t model, int n_vec, size_t* bytes);
vdc_status vdc_matvec_block(vdc_model_t model, double E, int n_vec, const int* parity,
                            const double* x, double* y, void* workspace, size_t ws_bytes,
                            void* stream);

/* Two-dimensional electron energy-loss spectrum (Eq. (17)) of solved
 * right-hand sides of the two-state model: for job k (eps_i, v_i, mu_i; host
 * vdc_job, model index 0) and its full-layout solution psi[k] (device complex
 * [n_jobs][psi_ld], psi_ld >= 2 Ng Nu, e.g. psi_out of vdc_solve), S_out[k][j]
 * (device double [n_jobs][n_grid]) = sum over every final state v_f of the
 * basis of this right-hand side's share of sigma_{v_f <- v_i} (Eq. (16) for
 * its mu_i, summed over mu_f; 0 for closed channels) times rho(loss_j -
 * (E_{v_f} - E_{v_i})), loss_j = loss0 + j dloss, rho a unit-area Gaussian of
 * full width at half maximum fwhm (eV; 0.010 in Sec. II.B).  The gerade and
 * ungerade parts are the jobs with mu_i = e and o; S is their sum.  Final
 * states farther than 8 standard deviations of rho from loss_j are skipped
 * (their weight is below 1e-13 of the peak).  Synchronises the stream. */
vdc_status vdc_eels_workspace_size(vdc_model_t model, int n_jobs, size_t* bytes);
vdc_status vdc_eels(vdc_model_t model, int n_jobs, const vdc_job* jobs, const double* psi,
                    size_t psi_ld, int n_grid, double loss0, double dloss, double fwhm,
                    double* S_out, void* workspace, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * The CO2-like three-state, four-mode model (Sec. III.C, the model class of
 * the e + CO2 paragraph): states sigma, Pi_x, Pi_y; modes s (symmetric
 * stretch), the bend (x, y) and a (asymmetric stretch); partial waves s,
 * p_x, p_y; H_0 = w_s (n_s+1/2) + w_b (n_x+n_y+1) + w_a (n_a+1/2) (Eq. (21));
 * U (Eq. (18) extended to second order):
 *   U_ss = E_sigma + k_sigma q_s + gs_sigma q_s^2 + gb_sigma (q_x^2+q_y^2) + ga_sigma q_a^2,
 *   U_xx, U_yy = E_pi + k_pi q_s + gs_pi q_s^2 + gb_pi (q_x^2+q_y^2) + ga_pi q_a^2
 *                +- c_rt (q_x^2 - q_y^2),   U_xy = 2 c_rt q_x q_y,
 *   U_sx = c_sp (1 + c_sp2 q_s) q_x,  U_sy = c_sp (1 + c_sp2 q_s) q_y;
 * discrete-continuum couplings f_d^mu(eps) O_d^mu with O_sigma^s = 1 + l_sigma q_s,
 * O_pix^s = h_pi q_x, O_piy^s = h_pi q_y, O_sigma^px = h_sigma q_x,
 * O_pix^px = O_piy^py = 1 + l_pi q_s, O_sigma^py = h_sigma q_y (others 0);
 * widths Gamma = A eps^(l+1/2) exp(-eps/B), l = 0 for the s wave, 1 for the
 * p waves, (A, B) per state class (sigma, pi) and wave class (s, p)
 * (Eq. (22)); level shift of Eq. (19); F as in Eq. (23).  All products of
 * q are products of truncated matrices.
 *
 * Every solve runs in one reflection sector (x -> -x, y -> -y): for the
 * right-hand side Phi^{v mu} the sector bits are px = (v_x + [mu = p_x]) & 1
 * and py = (v_y + [mu = p_y]) & 1.  Sector vectors hold one complex value per
 * grid point [n_s][n_a][n_x][n_y] (n_y fastest): at (n_x, n_y) the value is
 * the amplitude of sigma if (n_x + px, n_y + py) are both even, of Pi_x if
 * only n_x + px is odd, of Pi_y if only n_y + py is odd, and 0 if both are
 * odd. */
typedef struct {
  double omega_s, omega_b, omega_a;   /* > 0, eV                              */
  double E_sigma, E_pi;
  double k_sigma, k_pi;
  double gs_sigma, gb_sigma, ga_sigma, gs_pi, gb_pi, ga_pi;
  double c_rt, c_sp, c_sp2;
  double l_sigma, l_pi, h_sigma, h_pi;
  double A[2][2];            /* [state class sigma, pi][wave class s, p], >= 0   */
  double B[2][2];            /* the same, > 0                                    */
  int Ns, Nx, Ny, Na;        /* basis sizes: 1..1024, Ny 1..31                    */
  int hilbert_nodes;         /* 16..65536                                        */
  double hilbert_xmax;       /* > 0 eV                                            */
} vdc_co2_desc;

typedef struct vdc_co2* vdc_co2_t;   /* opaque */

/* One right-hand side: incident energy eps_i > 0, initial state v = (n_s,
 * n_x, n_y, n_a) in the basis, incoming partial wave mu_i (0 s, 1 p_x, 2 p_y). */
typedef struct {
  double eps_i;
  int v[4];
  int mu_i;
} vdc_co2_job;

vdc_status vdc_co2_create(const vdc_co2_desc* desc, vdc_co2_t* out);
vdc_status vdc_co2_destroy(vdc_co2_t model);

/* Workspace (device bytes) for vdc_co2_solve.  Host call, no device work.
 * With VDC_PREC_BLOCK it holds every job's block factor (the multipliers in
 * FP16 by columns and by rows, 1/D in FP32, and the factor kernel's band
 * staging: 8 (2 Ny + 1) + 64 bytes per grid point and job, 50 MB per job at
 * 24 x 24 x 24 x 8), so it grows with n_jobs; callers with less memory pass
 * fewer jobs per call. */
vdc_status vdc_co2_workspace_size(vdc_co2_t model, const vdc_solve_opts* opts, int n_jobs,
                                  const vdc_co2_job* jobs, size_t* bytes);

/* Solve (E - H_ef) Psi = Phi^{v mu} (Eqs. (26), (28)) for every job in one
 * persistent launch (after one launch for the level-shift tables of all
 * distinct energies, and with VDC_PREC_BLOCK one for the block factors):
 * with opts->method = VDC_COCG, FP64 COCG as described at vdc_method (the
 * paper's method for its CO2 model), else restarted FP64 GMRES(opts->restart) with right
 * preconditioning by the paper's block choice for this model class
 * (VDC_PREC_BLOCK: one block per (n_s, n_a) holding the bend plane, factored
 * once per job by complex-symmetric L D L^T without pivoting, formed in
 * FP32, stored with L in FP16 and 1/D in FP32, and applied in FP64 as the
 * exact inverse of the stored factor; a block with a vanishing pivot falls back to its diagonal; needs
 * Ny <= 24, else VDC_ERR_UNSUPPORTED), by the diagonal (VDC_PREC_JACOBI) or
 * by none,
 * until the FP64 true residual is <= tol ||Phi||.  opts->precision must be
 * VDC_FP64.  Then the amplitudes T[job][f][mu_f] = Phi^{v_f mu_f T} Psi
 * (Eq. (24)) for the finals (host int [n_final][4], states in the basis) and
 * the job's share of sigma (Eq. (16), summed over mu_f).
 * Outputs (device): T_out complex [n_jobs][n_final][3], sigma_out double
 * [n_jobs][n_final], psi_out complex [n_jobs][Ns*Na*Nx*Ny] sector vectors or
 * NULL; info host [n_jobs].  Synchronises the stream. */
vdc_status vdc_co2_solve(vdc_co2_t model, const vdc_solve_opts* opts, int n_jobs,
                         const vdc_co2_job* jobs, int n_final, const int* finals,
                         double* T_out, double* sigma_out, double* psi_out,
                         vdc_job_info* info, void* workspace, size_t ws_bytes, void* stream);

/* y = A x (which = 0) or y = M^{-1} x for the block preconditioner (which =
 * 1, the factor of vdc_co2_solve, Ny <= 24) at total energy E, on n_vec sector vectors (device complex
 * [n_vec][Ns*Na*Nx*Ny]), vector v in sector (sectors[2v], sectors[2v+1])
 * (host ints, 0/1).  For which = 0, entries of x at points that carry no
 * state (n_x + px and n_y + py both odd) are ignored and y is zero there, and
 * a non-finite entry of x may also reach y where its term carries a zero
 * weight.  x and y must not overlap.  Workspace: vdc_co2_ops_workspace_size().  Synchronises the
 * stream. */
vdc_status vdc_co2_ops_workspace_size(vdc_co2_t model, int n_vec, int which, size_t* bytes);
vdc_status vdc_co2_apply(vdc_co2_t model, double E, int which, int n_vec, const int* sectors,
                         const double* x, double* y, void* workspace, size_t ws_bytes,
                         void* stream);

/* ------------------------------------------------------------------------
 * The general model of the class, given by polynomial term lists (Sec. II.A-C
 * written for D discrete states, M vibrational modes and P partial waves;
 * the paper's CO2 model, Sec. III.C, is of this form with higher-order terms):
 *   H_0 = sum_k omega_k (n_k + 1/2)                                  (Eq. (21))
 *   U_dd' = e_state[d] delta_dd' + sum of U terms c prod_k q_k^p_k   (Eq. (18))
 *     (a U term names a pair (d, e) and adds to U_de and U_ed: U is symmetric)
 *   V_d^mu(eps) = f_d^mu(eps) O_d^mu, O_d^mu = sum of V terms (d, mu, c, p),
 *     2 pi (f_d^mu)^2 = Gamma_d^mu = A eps^(l + 1/2) exp(-eps/B)      (Eq. (22))
 *   F_dd' = sum_mu (O_d^mu)^T diag(F[f_d^mu f_d'^mu](E - E_nu)) O_d'^mu  (Eqs. (19), (23))
 *   A = E - H_0 - U - F,   Phi^{v mu}_d = f_d^mu(E - E_v) O_d^mu |v>  (Eqs. (25), (28))
 * with q_k = (a_k + a_k^+)/sqrt 2 truncated to the basis of mode k and every
 * monomial a product of truncated matrices.  Full vectors hold D blocks of
 * npts = prod_k nbasis[k] values, the block of state d at d * npts, point
 * index with the last mode fastest; N = D npts.
 * Limits: D <= 4, M <= 8, P <= 4, powers <= 4 per mode, nbasis 1..1024,
 * N <= 2^26; l belongs to the partial wave (equal for every state with
 * A > 0 on it), 0..4. */
#define VDC_MAX_STATES 4
#define VDC_MAX_MODES 8
#define VDC_MAX_WAVES 4
#define VDC_MAX_POWER 4

typedef struct {
  int d, e;                  /* U: the pair of states; V: state d, partial wave e */
  double coeff;              /* eV for U terms; dimensionless for V terms        */
  int pow[VDC_MAX_MODES];    /* power of q_k, 0..4 (0 past n_modes)             */
} vdc_term;

typedef struct {
  double A, B;               /* Gamma = A eps^(l+1/2) exp(-eps/B); A >= 0, B > 0 */
  int l;                     /* 0..4                                             */
} vdc_width;

typedef struct {             /* caller-owned; copied at creation                 */
  int n_states, n_modes, n_pw;
  const double* omega;       /* [n_modes] eV, > 0                                */
  const int* nbasis;         /* [n_modes]                                        */
  const double* e_state;     /* [n_states] eV                                    */
  int n_uterms;
  const vdc_term* uterms;
  int n_vterms;
  const vdc_term* vterms;
  const vdc_width* width;    /* [n_states][n_pw]; A = 0: no coupling            */
  int hilbert_nodes;         /* 16..65536                                        */
  double hilbert_xmax;       /* > 0 eV                                           */
  int dispatch;              /* non-zero: when the terms are exactly those of
                                vdc_model2d_desc (two states, modes g and u,
                                waves e and o), solve with the two-state
                                kernels (vdc_model_kind then reports 0)        */
} vdc_model_desc;

/* One right-hand side of a model built by vdc_model_create. */
typedef struct {
  double eps_i;              /* > 0                                              */
  int v[VDC_MAX_MODES];      /* initial vibrational state (0 past n_modes)       */
  int mu_i;                  /* incoming partial wave, 0..n_pw-1                 */
  int model;                 /* index into the call's models[]                   */
} vdc_mjob;

/* Build a model from term lists (host call; allocates its device tables).
 * The handle also serves vdc_model_destroy; the two-state entry points
 * (vdc_solve, vdc_matvec, ...) accept it only when vdc_model_kind is 0. */
vdc_status vdc_model_create(const vdc_model_desc* desc, vdc_model_t* out);

/* 0: the two-state kernels solve it (dispatch), 1: the term-list kernels. */
vdc_status vdc_model_kind(vdc_model_t model, int* kind);

/* Workspace bytes of vdc_model_solve (room for up to 64 finals).  Host call. */
vdc_status vdc_model_workspace_size(int n_models, const vdc_model_t* models,
                                    const vdc_solve_opts* opts, int n_jobs, const vdc_mjob* jobs,
                                    size_t* bytes);

/* Solve Eq. (26) for every job and project T and the sigma shares.  Models
 * of kind 0 go to vdc_solve (every option of it, including its FP64 re-solve
 * of FP32-inner jobs); models of kind 1 run one persistent launch (after
 * one launch for the level-shift planes of every distinct (model, E)): one
 * workgroup per job, COCG or restarted GMRES(restart) in complex FP64,
 * right-preconditioned by diag(A) (VDC_PREC_JACOBI) or not (VDC_PREC_NONE);
 * FP32_INNER, BLOCK and ROWS are VDC_ERR_UNSUPPORTED there.
 *   finals   host int [n_final][VDC_MAX_MODES] final states v_f
 *   T_out    device c16 [n_jobs][n_final][P], P = the largest n_pw of the
 *            models (kind 0: 2), T_{mu_f v_f <- mu_i v_i}, 0 for closed channels
 *   sigma_out device double [n_jobs][n_final]: the job's share of Eq. (16)
 *            (sum over mu_f); vdc_sum_partial_waves adds the mu_i shares
 *   psi_out  device c16 [n_jobs][max N] or NULL (full layout)
 *   info     host [n_jobs] or NULL.  Synchronises the stream. */
vdc_status vdc_model_solve(int n_models, const vdc_model_t* models, const vdc_solve_opts* opts,
                           int n_jobs, const vdc_mjob* jobs, int n_final, const int* finals,
                           void* workspace, size_t ws_bytes, double* T_out, double* sigma_out,
                           double* psi_out, vdc_job_info* info, void* stream);

/* y = A(E) x on n_vec full-layout vectors (device c16 [n_vec][N] each, not
 * overlapping) with the term-list kernels (any model from
 * vdc_model_create): the level-shift planes at E, then the two stencil
 * passes.  Kernel times by vdc_last_kernel_times.  Synchronises. */
vdc_status vdc_model_apply_workspace_size(vdc_model_t model, int n_vec, size_t* bytes);
vdc_status vdc_model_apply(vdc_model_t model, double E, int n_vec, const double* x, double* y,
                           void* workspace, size_t ws_bytes, void* stream);

/* The cross section of Eq. (16) summed over the incoming partial waves:
 * sigma[c][f] = sum over jobs j with collision[j] = c of share[j][f]
 * (shares from a solve call; jobs of one (eps_i, v_i) differ in mu_i),
 * added in job order.  collision: device int [n_jobs] (indices outside
 * 0..n_coll-1 are skipped); share: device double [n_jobs][n_final]; sigma:
 * device double [n_coll][n_final].  Asynchronous on the stream. */
vdc_status vdc_sum_partial_waves(int n_jobs, const int* collision, int n_coll, int n_final,
                                 const double* share, double* sigma, void* stream);

/* Thread-local text of the last error (never NULL). */
const char* vdc_last_error(void);

/* Library version string. */
const char* vdc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VDC_H */
