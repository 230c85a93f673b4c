/*
 * fftnk.h -- C-ABI of libfftnk, an MI355X (gfx950) implementation of the hot
 * path of the finite-strain FFT-based Newton-Krylov homogenisation solver of
 * T.W.J. de Geus, J. Vondrejc, J. Zeman, R.H.J. Peerlings, M.G.D. Geers,
 * "Finite strain FFT-based non-linear solvers made simple", CMAME 318 (2017).
 *
 * Conventions (all entry points)
 * ------------------------------
 *  - Grid: a periodic cell of n0 x n1 x n2 voxels; grid axis d is the reference
 *    direction X_{d+1}.  n = n0*n1*n2.
 *  - Tensor fields are device arrays, component-major [9][n0][n1][n2] (axis a2
 *    fastest), component c = 3*i + j holds A_ij, F_ij = dx_i/dX_j (paper's
 *    nomenclature appendix).  A batched context concatenates the RVE blocks in
 *    RVE order: RVE r starts at element 9*(n_0 + ... + n_{r-1}).
 *  - F, P and the homogenised stresses are always FP64.  Fields passed to
 *    fftnk_project / fftnk_apply_operator use the context precision
 *    (FFTNK_FP64: double, FFTNK_FP32_MIXED: float).
 *  - Device memory is owned by the caller.  The context never allocates device
 *    memory: all of its state lives in one caller-provided workspace (see
 *    fftnk_workspace_bytes / fftnk_bind_workspace) and is never freed by it.
 *    Host arrays are read (or written) during the call only.
 *  - All work is enqueued on the HIP stream given at creation; calls that
 *    return host results synchronise that stream before returning.
 *  - Every call returns an int status (FFTNK_OK = 0) and never throws.
 *  - A context is not thread safe; calls on one context must not overlap.
 */
#ifndef FFTNK_H
#define FFTNK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
enum {
  FFTNK_OK = 0,
  FFTNK_EINVAL = 1,          /* bad argument (size, pointer, tolerance, parameters)          */
  FFTNK_ESTATE = 2,          /* call order: workspace / phases / material not set            */
  FFTNK_ENOMEM = 3,          /* workspace smaller than fftnk_workspace_bytes                 */
  FFTNK_EHIP = 4,            /* a HIP runtime call failed                                     */
  FFTNK_ECG_MAXIT = 5,       /* CG reached max_cg iterations without convergence            */
  FFTNK_ECG_BREAKDOWN = 6,   /* CG found <p, A p> <= 0 or non-finite (indefinite tangent)    */
  FFTNK_ENEWTON_MAXIT = 7,   /* Newton reached max_newton solves without convergence        */
  FFTNK_ENONFINITE = 8,      /* NaN / Inf in the load, the iterate or a residual             */
  FFTNK_EMATERIAL = 9,       /* constitutive update failed (e.g. return mapping)             */
  FFTNK_EUNSUPPORTED = 10    /* grid length or configuration not supported by the kernels   */
};

/* precision of the Krylov solve (the Newton residual, F, P are always FP64) */
enum { FFTNK_FP64 = 0, FFTNK_FP32_MIXED = 1 };

/* material models */
enum { FFTNK_SVK = 0, FFTNK_J2 = 1 };

#define FFTNK_MAX_SOLVES 64

/* statistics of one load increment of one RVE */
typedef struct {
  int status;                              /* FFTNK_* of this RVE                          */
  int n_solves;                            /* linear solves (the boundary-condition solve included) */
  int cg_iters[FFTNK_MAX_SOLVES];          /* CG iterations (operator applications) per solve */
  double newton_res[FFTNK_MAX_SOLVES];     /* ||dF|| / ||F_t + dFbar|| after each solve    */
  double cg_relres[FFTNK_MAX_SOLVES];      /* final recursive ||r|| / ||b|| of each solve   */
  double t_ms;                             /* wall time of the call                          */
} fftnk_stats;

typedef struct fftnk_ctx fftnk_ctx;

/*
 * Create a context for one periodic cell of n0 x n1 x n2 voxels (n0, n1 in
 * 2..512, n2 in 2..256; any factorisation: radices 2, 3, 4, 5, 7, 8 run as
 * register butterflies, other primes as direct sums).  A plane-strain cell
 * (the paper's 2-D example) is an n0 x n1 x 2 cell whose phases do not vary
 * along a2 and whose Fbar has F33 = 1, F13 = F23 = F31 = F32 = 0: its fields
 * have no a2 frequency but zero, so xi_2 = 0 and G acts as the 2-D projection.  precision: FFTNK_FP64 or
 * FFTNK_FP32_MIXED.  hip_stream: a hipStream_t (NULL = default stream).
 * Returns FFTNK_EINVAL for bad sizes.  The context owns host memory only;
 * creation makes no HIP call.
 */
int fftnk_create(fftnk_ctx** out, int n0, int n1, int n2, int precision, void* hip_stream);

/*
 * Create a context for nrve independent cells solved together (batching
 * pattern); dims is a host array [nrve][3].  Each RVE has its own load,
 * Newton and CG state; every kernel launch covers all RVEs.
 */
int fftnk_create_batched(fftnk_ctx** out, int nrve, const int* dims, int precision, void* hip_stream);

/* Bytes of device workspace the context needs (256-byte aligned start). */
size_t fftnk_workspace_bytes(const fftnk_ctx* ctx);

/*
 * Instrumentation: the context's launch geometry as one JSON object (per cell:
 * sizes, offsets, grid lines per a2 work-group, pencils per column
 * work-group, work-groups per launch kind, and per axis the radix plan and
 * the FFT engine: 8 or 12 points per thread in registers, 0 the LDS engine;
 * per context: work-groups per launch kind, LDS bytes per kernel family,
 * workspace bytes, the plan policy and the partial-sum stride).  Writes a NUL-terminated string into buf (host, len
 * bytes); *needed (optional) receives the length it needs; FFTNK_ENOMEM when
 * len is smaller.  Makes no HIP call: a context can be created and described
 * without a GPU (creation allocates host memory only; the host staging
 * buffer and the capture stream come with fftnk_bind_workspace).
 */
int fftnk_describe(const fftnk_ctx* ctx, char* buf, size_t len, size_t* needed);

/*
 * FFT plan policy of a context: which engine and tile size each pass uses
 * (the transforms of Sec. 2.5 are the same under every policy; results differ
 * by rounding order only).  Bit fields of `policy`:
 *   bits 0-2  axis d (a0, a1, a2) on the LDS engine even where its length has
 *             a register-resident engine;
 *   bits 3-4  s in 0..2: the LDS-engine a1 / a0 passes take at most 8 >> s
 *             (FP64) or 16 >> s (FP32) pencils per work-group (3 is invalid);
 *   bit 5     the register-engine a2 passes take half their default grid
 *             lines per work-group.
 * 0 is the default.  May be called before or after fftnk_bind_workspace (the
 * workspace is sized for every policy); drops the captured CG graphs.
 * FFTNK_EINVAL for an invalid code, FFTNK_EUNSUPPORTED when a kernel's LDS
 * budget would be exceeded (the context keeps its policy).  The policy in use
 * is reported by fftnk_describe ("policy").
 */
int fftnk_set_plan(fftnk_ctx* ctx, unsigned policy);

/*
 * Autotuner: times one operator application (the tangent at the committed
 * state F_t applied to a zero field; every pass of the CG operator) under
 * every policy that changes the context's launches, `reps` back-to-back
 * applications, best of three rounds, and keeps the fastest.  The choice is
 * cached per process under the context's precision, material model, Nyquist
 * choice and cell sizes; with use_cache != 0 a cached choice is applied
 * without timing (*ms = -1).  Needs a bound workspace, phases and material
 * (else FFTNK_ESTATE); overwrites the CG vectors x, p, w and the spectrum
 * (scratch between calls).  *policy (optional) receives the policy applied,
 * *ms (optional) its milliseconds per application.  reps in 1..1000.  On a
 * HIP error the previous policy is restored.  Synchronous.
 */
int fftnk_autotune(fftnk_ctx* ctx, int reps, int use_cache, unsigned* policy, double* ms);

/*
 * Hand the context its workspace: dev must stay valid until the context is
 * destroyed or rebound.  Resets the state to F_t = I (stress-free start,
 * Algorithm 1's initialisation).  FFTNK_ENOMEM if bytes is too small.
 */
int fftnk_bind_workspace(fftnk_ctx* ctx, void* dev, size_t bytes);

/* Phase index per voxel (device uint8 [n]; batched: concatenated).  Copied. */
int fftnk_set_phases(fftnk_ctx* ctx, const uint8_t* phase_dev);

/*
 * Material (paper Sec. 4.2 for FFTNK_SVK: S = C:E, E = (F^T F - I)/2,
 * P = F S with isotropic C from bulk modulus K and shear modulus mu,
 * lambda = K - 2 mu/3; Sec. 5 for FFTNK_J2: F = Fe Fp, Kirchhoff stress
 * tau = C : ln(be)/2, von Mises yield with linear hardening
 * tau_y = tau_y0 + H eps_p, exponential-map return mapping, P = tau F^-T).
 * params_host holds, per phase, {K, mu} for SVK and {K, mu, tau_y0, H} for
 * J2.  nphase <= 256 (a batch may give every cell its own phases).  J2 needs
 * an FFTNK_FP64 context (else FFTNK_EUNSUPPORTED); a point whose return
 * mapping fails (det F <= 0) makes the increment fail with FFTNK_ENONFINITE.
 */
int fftnk_set_material(fftnk_ctx* ctx, int model, int nphase, const double* params_host);

/*
 * Optional per-voxel shear modulus mu(x) (device double [n]; copied) that
 * replaces the phase value of mu; K stays per phase.  NULL switches it off.
 */
int fftnk_set_modulus_field(fftnk_ctx* ctx, const double* mu_dev);

/*
 * Options: FFTNK_OPT_GRAPHS (1 = replay CG iterations from captured HIP graphs,
 * the default; 0 = launch every kernel), FFTNK_OPT_CHECK_EVERY (CG iterations
 * between two host checks of the convergence flags, 1..64, default 4).  Both
 * change timing only, never results.
 * FFTNK_OPT_NYQUIST selects the value of G-hat at the Nyquist frequencies of
 * even axes (App. C): 0 (default) zero there, which keeps F compatible; 1 the
 * identity there, which keeps the stress equilibrated.  It applies to every
 * cell and to every later call (projection, operator, solves, adjoint).  With
 * 1 the operator acts on the Nyquist rotations F W (W skew) through the
 * geometric stiffness only: singular at F = I and indefinite wherever the
 * stress has a compressive direction, so CG may end in FFTNK_ECG_BREAKDOWN
 * (typically under shear), and it converges more slowly under tension.
 * Values other than 0 / 1 give FFTNK_EINVAL.
 * FFTNK_OPT_GMRES_RESTART (1..256) reserves the Arnoldi basis of restarted
 * GMRES (m + 1 vector fields of the context precision) in the workspace: set
 * it after creation and before fftnk_workspace_bytes / fftnk_bind_workspace
 * (afterwards FFTNK_ESTATE); it enables FFTNK_KRYLOV_GMRES.
 * FFTNK_OPT_J2_TANGENT (0 default, 1): for the J2 law (Sec. 5) in FP64, 1
 * stores the parts of the consistent tangent that do not depend on the
 * direction (eigenbasis of the trial elastic left Cauchy-Green tensor, the
 * principal algorithmic moduli, the principal Kirchhoff stresses; 24 doubles
 * per voxel, reserved in the workspace) once per linearisation point, instead
 * of redoing the return mapping and eigen-decomposition at every operator
 * application.  Same results up to rounding order.  Set it before
 * fftnk_workspace_bytes / fftnk_bind_workspace (afterwards FFTNK_ESTATE).
 * FFTNK_OPT_X_WINDOW (1..8, default 8): the CG of Sec. 2.6 keeps the search
 * directions of this many iterations (W vector fields of the context
 * precision in the workspace) and adds their steps alpha_j p_j to the iterate
 * x once every W iterations, in the order of j, instead of reading and
 * writing x at every iteration; the same roundings, so the same results for
 * every W.  1 keeps one direction and updates x at every iteration.  Set it
 * before fftnk_workspace_bytes / fftnk_bind_workspace (afterwards
 * FFTNK_ESTATE).
 */
enum { FFTNK_OPT_GRAPHS = 1, FFTNK_OPT_CHECK_EVERY = 2, FFTNK_OPT_NYQUIST = 3, FFTNK_OPT_GMRES_RESTART = 4,
       FFTNK_OPT_J2_TANGENT = 5, FFTNK_OPT_X_WINDOW = 6 };
int fftnk_set_option(fftnk_ctx* ctx, int option, int value);

/* F_t := I (and virgin history): the start state of Algorithm 1. */
int fftnk_reset_state(fftnk_ctx* ctx);

/*
 * Krylov method of every later linear solve.  Sec. 2.6 uses conjugate
 * gradients as one choice of projection-based Krylov solver;
 * FFTNK_KRYLOV_CG (the default) is that.  FFTNK_KRYLOV_CHEBYSHEV and
 * FFTNK_KRYLOV_RICHARDSON are the classical fixed-coefficient alternatives
 * on the same operator and the same fused kernels: with bounds 0 < lo < hi
 * (Richardson: lo <= hi) of the spectrum of A on range(G),
 *   Chebyshev (Saad, Iterative Methods for Sparse Linear Systems, Sec. 12.1):
 *     x += gamma_k p_k, r -= gamma_k A p_k, p_{k+1} = r_{k+1} + beta_{k+1} p_k
 *     with gamma, beta from the three-term recurrence of Chebyshev
 *     polynomials on [lo, hi];
 *   Richardson: x += omega r, r -= omega A r, omega = 2 / (lo + hi).
 * They need no inner product but the stopping test's <r, r>.  Bounds that do
 * not enclose the spectrum make them diverge (the solve then ends with
 * FFTNK_ENONFINITE or FFTNK_ECG_MAXIT).  At F = I on gradients,
 * mu_min <= <p, A p> / <p, p> <= 3 K_max (periodic Korn inequality and the
 * largest local eigenvalue); finite strain and plasticity move the spectrum.
 * FFTNK_KRYLOV_GMRES: restarted GMRES(m) (Saad, same book, Alg. 6.9; Arnoldi
 * with classical Gram-Schmidt, repeated where the first pass cancels more than
 * the Daniel-Gragg-Kaufman-Stewart test allows, Givens rotations, m from
 * FFTNK_OPT_GMRES_RESTART, else FFTNK_ESTATE; lo, hi unused), for tangents
 * that are not symmetric; it needs no bounds but stores m + 1 basis fields
 * and synchronises with the host once per inner-product batch.
 * Same stopping test as CG (GMRES: on its least-squares residual); the counts
 * reported as cg_iters are operator applications.  Bad method or bounds:
 * FFTNK_EINVAL.
 */
enum { FFTNK_KRYLOV_CG = 0, FFTNK_KRYLOV_CHEBYSHEV = 1, FFTNK_KRYLOV_RICHARDSON = 2, FFTNK_KRYLOV_GMRES = 3 };
int fftnk_set_krylov(fftnk_ctx* ctx, int method, double lo, double hi);

/*
 * One load increment of Algorithm 1 (Sec. 3.1-3.2) with the macroscopic
 * deformation gradient prescribed: dFbar = Fbar - mean(F_t); the first solve
 * G:K(F_t):dF = -G:K(F_t):dFbar distributes the load with the tangent of the
 * start state, then Newton iterations G:K(F_i):dF = -G:P(F_i) until
 * ||dF|| / ||F_t + dFbar|| < eta_nw (and at least two solves).  Each linear
 * system is solved by CG to ||r|| <= eta_cg ||b|| (FP32_MIXED: at least 1e-6).
 *
 * Fbar_host [nrve][9]; F_dev, P_dev (optional, may be NULL): device double
 * [9][n] receiving the converged F and P; Pbar_host [nrve][9] receives the
 * voxel mean of P; stats (optional) [nrve].  On success the converged state is
 * committed as the new F_t.  On any failure the committed state is unchanged
 * and the outputs are undefined.
 */
int fftnk_solve_increment(fftnk_ctx* ctx, const double* Fbar_host, double eta_nw, double eta_cg, int max_newton,
                          int max_cg, double* F_dev, double* P_dev, double* Pbar_host, fftnk_stats* stats);

/*
 * One load increment under mixed macroscopic control.  Not in the paper: its
 * Sec. 3.1 prescribes the whole macroscopic deformation gradient and leaves
 * stress or mixed control to the literature; this builds it from the same
 * boundary-condition system and operator.
 *
 * Per RVE r, components k with mask_host[9r+k] != 0 prescribe the homogenised
 * stress, Pbar_k = Ptarget_host[9r+k]; the others prescribe Fbar_k =
 * Fbar_host[9r+k].  Fbar_host's masked entries are the starting guess (e.g.
 * the previous increment's values) and receive the solution (in/out, host
 * [nrve][9]).  Outer Newton iteration on the masked entries: each pass solves
 * the deformation-controlled increment of fftnk_solve_increment at the current
 * Fbar (the first from the committed state, later ones from the previous
 * pass's equilibrium); it stops when max_k |Pbar_k - Ptarget_k| <= tol_stress
 * (absolute, stress units) over the masked k; otherwise the masked block of
 * the macroscopic tangent (fftnk_macro_tangent, at the current equilibrium,
 * its columns solved to CG tolerance max(eta_cg, 1e-4): the block only steers
 * the step) gives the Newton step of Fbar.  outer_host (optional, [nrve]) receives the
 * passes taken; stats (optional, [nrve]) lists every linear solve in order
 * (Newton and tangent solves; n_solves counts them all, the arrays hold the
 * first FFTNK_MAX_SOLVES).  The remaining arguments and the commit / failure
 * rules are those of fftnk_solve_increment; in addition FFTNK_ENEWTON_MAXIT
 * when max_outer passes do not reach tol_stress, and FFTNK_EINVAL when the
 * masked tangent block is singular (the mask leaves a direction of Fbar with
 * no stress response, e.g. rigid rotations with all nine components
 * prescribed at zero stress).
 */
int fftnk_solve_increment_mixed(fftnk_ctx* ctx, double* Fbar_host, const int* mask_host, const double* Ptarget_host,
                                double tol_stress, int max_outer, double eta_nw, double eta_cg, int max_newton,
                                int max_cg, double* F_dev, double* P_dev, double* Pbar_host, fftnk_stats* stats,
                                int* outer_host);

/*
 * Macroscopic (homogenised) tangent at the last committed state: C_host
 * [nrve][9][9] receives C[r][i][m] = dPbar_i / dFbar_m for every column m with
 * want_host[9r+m] != 0 (want_host NULL: all nine), zeros elsewhere.  A unit
 * macroscopic increment E_m spreads as E_m + dF with the boundary-condition
 * solve of Sec. 3.1, G:K(F_t):dF = -G:K(F_t):E_m; with A w = G(K(F_t):E_m)
 * (one CG per column, all RVEs together), column m = mean(K(F_t) : (E_m - w)).
 * Not in the paper.  CG parameters as in fftnk_solve_increment; stats
 * (optional, [nrve]) lists one solve per column.
 */
int fftnk_macro_tangent(fftnk_ctx* ctx, const int* want_host, double eta_cg, int max_cg, double* C_host,
                        fftnk_stats* stats);

/*
 * Linearisation point of fftnk_apply_operator: F (device double [9][n]) is
 * copied into the context (and rounded to float in FP32_MIXED mode).
 */
int fftnk_set_linearization(fftnk_ctx* ctx, const double* F_dev);

/*
 * The projected-tangent operator (Sec. 2.6, eq. iter:system; Sec. 4.3):
 * Ap = G( K(F) : p ), with the St. Venant-Kirchhoff tangent action
 * dP = p S + F [lambda tr(F^T p) I + mu (F^T p + p^T F)] recomputed per voxel
 * from the linearisation point F.  p, Ap: device [9][n] in context precision;
 * they must not alias.
 */
int fftnk_apply_operator(fftnk_ctx* ctx, const void* p_dev, void* Ap_dev);

/*
 * One linear solve A x = G(b) with the operator of fftnk_apply_operator at the
 * linearisation point of fftnk_set_linearization, x0 = 0, by the Krylov method
 * of fftnk_set_krylov (CG by default), stopped when ||r|| <= eta ||G(b)||
 * (FFTNK_FP32_MIXED: eta at least 1e-6) or after max_it operator
 * applications (FFTNK_ECG_MAXIT, x then holds the last iterate).  b_dev,
 * x_dev: device double [9][n] (b is projected with G in FP64 first; in FP32
 * mode x is the FP32 solution rounded up and projected again).  stats
 * (optional, [nrve]): one solve with its iteration count and final
 * ||r|| / ||G(b)||.  Batched contexts solve every RVE together.
 */
int fftnk_solve_linear(fftnk_ctx* ctx, const double* b_dev, double* x_dev, double eta, int max_it,
                       fftnk_stats* stats);

/*
 * The compatibility projection alone (Sec. 2.5; App. C for even axes):
 * Ga = Re F^-1[ G-hat : F(a) ], (G-hat : A-hat)_ij = xi_j (sum_l xi_l A-hat_il)/|xi|^2,
 * zero at k = 0 and on every even axis' Nyquist index (the identity there
 * with FFTNK_OPT_NYQUIST = 1).  a, Ga: device
 * [9][n] in context precision; may alias.
 */
int fftnk_project(fftnk_ctx* ctx, const void* a_dev, void* Ga_dev);

/*
 * Constitutive update alone: P = P(F) per voxel (device double [9][n]) and
 * the voxel mean Pbar_host [nrve][9].  For J2 the history of the last
 * committed state is used and not modified.
 */
int fftnk_constitutive(fftnk_ctx* ctx, const double* F_dev, double* P_dev, double* Pbar_host);

/*
 * Adjoint sensitivity of the homogenised stress at the last committed state
 * (not in the paper; derived from its boundary-condition system, Sec. 3.1,
 * and the symmetry of G, Sec. 2.3).  For each RVE r with cotangent
 * g_r = dL/dPbar_r (gbar_host [nrve][9]) one CG solve with the same operator
 * at F_t gives the adjoint field w in range(G): A w = G(K(F_t) : g_r); then per
 * voxel  dL/dmu(x) = (1/n)(g_r - w(x)) : F.2dev(E)  and
 *        dL/dK(x)  = (1/n)(g_r - w(x)) : tr(E) F.
 * dLdmu_dev / dLdK_dev (device double [n], batched: concatenated per RVE;
 * dLdK_dev may be NULL) are overwritten.  Parameters of the CG as in
 * fftnk_solve_increment; stats (optional) [nrve] gets one solve per RVE.
 */
int fftnk_adjoint(fftnk_ctx* ctx, const double* gbar_host, double eta_cg, int max_cg, double* dLdmu_dev,
                  double* dLdK_dev, fftnk_stats* stats);

/*
 * Instrumentation: enqueue pass `pass` (1..5) of the projected-tangent
 * operator alone, on the context's internal buffers (pass 1 reads the internal
 * direction field and the linearisation point, pass 5 writes the internal
 * result field), without synchronising.  The passes are: 1 tangent action and
 * a2 forward transform, 2 a1 forward, 3 a0 forward + projection + a0 inverse,
 * 4 a1 inverse, 5 a2 inverse.  For timing a single kernel with stream events;
 * results are meaningful only when the five run in order.
 */
int fftnk_launch_pass(fftnk_ctx* ctx, int pass);

/*
 * Instrumentation: time each kernel of a CG iteration (Sec. 2.6) at the
 * current iterate.  The right-hand side is -G(P) of the current iterate's
 * stress (so call it after a solve); the CG runs with tolerance 0 and no
 * iteration cap: W + 1 whole iterations untimed (W = FFTNK_OPT_X_WINDOW), then
 * max(iters, W) whole iterations with pass 1 between two stream events, in
 * place (it reads what the iteration before wrote), then every other kernel
 * `iters` times back to back between two events (the context's Krylov vectors
 * are clobbered, the committed state is not).  ms_host[8] (host) receives the mean time of
 * one launch of: 0 pass 1 (p update, tangent action, a2 forward) at an
 * iteration inside a window, 1 alpha (0: its work-groups run in pass 2's
 * launch and are timed with it), 2 pass 2, 3 pass 3, 4 pass 4, 5 pass 5 (a2
 * inverse, residual update), 6 beta, 7 pass 1 at an iteration that applies the
 * window of x updates (W = 1: every iteration; then 0 and 7 agree).
 * 1 <= iters <= 10000.  FFTNK_ESTATE if a cell's right-hand side is zero
 * (nothing to iterate on); synchronises.
 */
int fftnk_profile_cg(fftnk_ctx* ctx, int iters, double* ms_host);

/*
 * Instrumentation, independent of any context: the achievable HBM streaming
 * rate of the device, the ceiling for passes that move each byte of their
 * working set once (every pass of the operator does; Sec. 3.3 names the
 * transforms as the cost, and on this device they are bound by memory).
 * kind: FFTNK_STREAM_READ (sum of src1, one partial per work-group written to
 * the first doubles of dst), _WRITE (fill dst), _COPY (dst = src1), _TRIAD
 * (dst = src1 + 0.5 src2); lane_bytes 8 or 16 (double or double2 accesses);
 * kind | FFTNK_STREAM_NONTEMPORAL: every load and store non-temporal.
 * dst, src1, src2: caller-owned device buffers of `bytes` bytes each (src1 /
 * src2 may be NULL where the kind does not read them); bytes a multiple of
 * lane_bytes.  One untimed launch, then `reps` (1..10000) back-to-back
 * launches between two events on hip_stream (NULL: the default stream);
 * ms_host receives the mean ms per launch.  Bytes moved per launch: read,
 * write: bytes; copy: 2 bytes; triad: 3 bytes.  Synchronises the stream.
 * FFTNK_EINVAL on a bad kind, lane width, size, count or missing pointer.
 */
/*
 * The projection of fftnk_project without a context and without any
 * allocation, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels (G-hat zero at Nyquist frequencies, default FFT plan), with the
 * spectrum and launch tables in one statically allocated device buffer of
 * 64 MiB per GPU that the library holds until the process ends.  a_dev /
 * Ga_dev: caller-owned device fields [9][n0][n1][n2] of double (FFTNK_FP64)
 * or float (FFTNK_FP32_MIXED); hip_stream: a stream of the current device
 * (NULL: its default stream).  Cells whose spectrum and tables exceed the
 * buffer (e.g. FP64 beyond about 96^3, FP32 beyond about 120^3) return
 * FFTNK_ENOMEM; lengths as in fftnk_create.  The first call on a device, and
 * every call whose grid or precision differs from the previous call's on that
 * device, uploads the tables and synchronises the stream; other calls only
 * enqueue.  All calls on one GPU share its buffer: calls that overlap in time
 * on one GPU (other streams, other host threads between enqueue and
 * completion) race.  Not capturable while the tables are uploaded (the first
 * call on a device, or a change of grid or precision).
 */
int fftnk_project_noalloc(int n0, int n1, int n2, int precision, const void* a_dev, void* Ga_dev, void* hip_stream);

enum { FFTNK_STREAM_READ = 0, FFTNK_STREAM_WRITE = 1, FFTNK_STREAM_COPY = 2, FFTNK_STREAM_TRIAD = 3,
       FFTNK_STREAM_NONTEMPORAL = 16 };
int fftnk_stream(int kind, int lane_bytes, void* dst, const void* src1, const void* src2, size_t bytes, int reps,
                 void* hip_stream, double* ms_host);

/*
 * Checkpoint of the J2 history (Alg. 1, "store history variables"): device
 * double [7][n] -- C_p^-1 as xx yy zz xy yz xz, then the accumulated plastic
 * strain; batched: each of the 7 planes holds all RVEs in order.  Virgin state
 * (after bind / reset): C_p^-1 = I, eps_p = 0.
 */
int fftnk_get_history(fftnk_ctx* ctx, double* hist_dev);
int fftnk_set_history(fftnk_ctx* ctx, const double* hist_dev);

/* Checkpoint: copy out / in the committed F_t (device double [9][n]). */
int fftnk_get_state(fftnk_ctx* ctx, double* F_dev);
int fftnk_set_state(fftnk_ctx* ctx, const double* F_dev);

/* Human-readable name of a status code (static string). */
const char* fftnk_status_string(int status);

/* Release the context's host memory (the workspace stays the caller's). */
void fftnk_destroy(fftnk_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* FFTNK_H */
