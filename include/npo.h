/*
 * npo.h -- C ABI of the MI355X hot path of the nonlinear-optimal-perturbation
 * (NLOP) method for pulsatile pipe flow: Keuchel & Avila, "Nonlinear optimal
 * perturbation growth in pulsatile pipe flow", arXiv 2509.10103.
 *
 * Conventions shared by every call
 * --------------------------------
 * Units are the paper's (Sec. 2): lengths in pipe radii, velocities in twice
 * the mean bulk velocity, time in radius / (2 x bulk velocity).  The laminar
 * flow is the Sexl-Womersley profile with bulk velocity
 * u_b(t) = 1/2 [1 + A sin(2 pi t / T)], T = 2 pi Re / Wo^2 (Sec. 2).
 *
 * A "field" is a complex128 array [3][nr][M+1][2K+1] (interleaved re/im
 * doubles) in device memory: components (u_r, u_theta, u_z), radial node j
 * (r_j ascending, r_{nr-1} = 1 is the wall), azimuthal index m = 0..M and axial
 * index kk in FFT order (k = 0..K, -K..-1), with M = (ntheta-1)/3 and
 * K = (nz-1)/3 so that the ntheta x nz physical grid is the 3/2-rule
 * dealiasing grid of the Fourier-Galerkin expansion (Sec. 2.3).  The m = 0
 * column is a Hermitian series in k.  Inner products are the discrete form of
 * the paper's volume integral <.> (Sec. 2):
 *   <a,b>_W = 2 pi L_z sum_{k,m} c_m sum_j w_j Re(conj(a) . b), c_0 = 1, c_m = 2.
 *
 * Ownership: the caller owns every device buffer passed in (fields, the
 * workspace, the checkpoint arena, device scalars).  A plan owns only its
 * constant device tables, allocated by npo_plan_create and released by
 * npo_plan_destroy.  After plan creation, device memory is allocated only by
 * (a) the first sweep of a workspace with step graphs enabled (the HIP runtime
 * instantiates the captured graphs; the plan also creates its capture stream
 * once), (b) the batch calls (device descriptor tables and a capture stream,
 * owned by the batch and released by npo_batch_destroy) and (c)
 * npo_profile_begin (HIP events); every other call allocates nothing.
 *
 * Asynchrony: every call that takes `stream` (a hipStream_t; NULL is the
 * default stream) only enqueues work on that stream unless stated otherwise;
 * outputs are valid once the stream reaches that point.  Calls that return a
 * host scalar say so and synchronise the stream.
 *
 * Errors: argument and shape errors return synchronously (NPO_EINVAL,
 * NPO_EUNSUPPORTED) before anything is enqueued; launch and runtime errors
 * return NPO_EHIP.  npo_last_error() gives a message for the calling thread.
 *
 * Tracing: with NPO_TRACE=1 in the environment the plan, sweep, iteration and
 * batch calls open roctx ranges (rocprofv3 --marker-trace shows them).
 */
#ifndef NPO_H
#define NPO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t npo_status;
#define NPO_OK            0
#define NPO_EINVAL       -1   /* bad argument or size                           */
#define NPO_ENOMEM       -2   /* plan tables could not be allocated              */
#define NPO_EHIP         -3   /* a HIP runtime or launch error                   */
#define NPO_EUNSUPPORTED -4   /* grid outside the sizes the kernels support      */
#define NPO_ESTATE       -5   /* call out of order (e.g. no forward sweep yet)   */

/* Grid: nr radial nodes (8..64), ntheta and nz physical points (products of 2
 * and 3, ntheta in 6..128, nz even in 6..2048), pipe length lz in radii. */
typedef struct { int32_t nr, ntheta, nz; double lz; } npo_grid;
/* Flow: Re (diameter and mean bulk velocity), Womersley number Wo, pulsation
 * amplitude A = U_max/U_bar - 1 (Sec. 1). A = 0 is steady Hagen-Poiseuille. */
typedef struct { double re, wo, amp; } npo_flow;
/* Time: step dt, initial time tau0 (the perturbation is introduced at t0,
 * Sec. 2), horizon nsteps (the gain is evaluated at tau0 + nsteps*dt) and the
 * number of corrector passes of the predictor-corrector step (1..3; 2 keeps
 * the explicit convective terms stable at axial CFL numbers up to ~2). */
typedef struct { double dt, t0; int64_t nsteps; int32_t ncorr; } npo_time;

typedef struct npo_plan_s* npo_plan;

typedef struct {
    int32_t nr, ntheta, nz, M, K, nk;   /* nk = 2K+1                              */
    int64_t field_elems;                /* complex elements per field = 3*nr*(M+1)*nk */
    int64_t field_bytes;                /* 16 * field_elems                       */
    int64_t workspace_bytes;            /* device workspace every run call needs  */
    int64_t scalars_bytes;              /* device scalar block for npo_iterate    */
    double period, k0, dt, t0;
    int64_t nsteps;
} npo_info;

/* Message describing the last error on this thread ("" if none). */
const char* npo_last_error(void);

/* Build a plan: radial nodes r_j = cos(pi (nr-1-j)/(2 nr-1)), quadrature
 * weights w_j (interpolatory in r^2), sixth-order 7-point FD weights with
 * parity folding at the axis and one-sided wall rows (Sec. 2.3), Womersley
 * profile tables (Sec. 2), FFT twiddles.  Allocates the plan's device tables
 * on the current device.  flags must be 0. */
npo_status npo_plan_create(const npo_grid* grid, const npo_flow* flow, const npo_time* time,
                           uint32_t flags, npo_plan* out);
npo_status npo_plan_destroy(npo_plan plan);
npo_status npo_plan_info(npo_plan plan, npo_info* out);

/* Host copies of the plan's radial tables: r[nr], w[nr], and the FD weights
 * D1[2][nr][7], D2[2][nr][7] (parity index 0 = even, 1 = odd) acting on the
 * nodes col0[j] .. col0[j]+6.  Any pointer may be NULL. */
npo_status npo_plan_tables(npo_plan plan, double* r, double* w, double* D1, double* D2, int32_t* col0);

/* Laminar Sexl-Womersley flow at time t (Sec. 2, base flow driven at bulk
 * velocity u_b(t)): U_dev[j] = U(r_j, t) and dUdr_dev[j] = dU/dr(r_j, t)
 * (= -Omega_theta), j = 0..nr-1, written by a kernel on `stream` into caller
 * device arrays of nr doubles.  t is in the solver's time units (absolute,
 * not relative to t0).  NPO_EINVAL for a null pointer or non-finite t. */
npo_status npo_base_flow(npo_plan plan, double t, double* U_dev, double* dUdr_dev, void* stream);

/* Pieces of the step, exposed for testing each kernel (all device pointers,
 * workspace ws of workspace_bytes):
 *   npo_nonlinear:     out = P_K F[u x w] + U x w + u x Om at time t, w = curl u
 *                      (dealiased convective term, Sec. 2 direct equations);
 *   npo_nonlinear_adj: out = W-adjoint of the tangent of the above at u, applied to y;
 *   npo_solve:         out = S(R): H out + grad p = R, div out = 0, out(1) = 0,
 *                      with zero flux for the mean mode (Sec. 2.3);
 *   npo_solve_adj:     out = W-adjoint of S applied to y. */
npo_status npo_nonlinear(npo_plan plan, void* ws, const void* u, double t, void* out, void* stream);
npo_status npo_nonlinear_adj(npo_plan plan, void* ws, const void* u, double t, const void* y,
                             void* out, void* stream);
npo_status npo_solve(npo_plan plan, void* ws, const void* R, void* out, void* stream);
npo_status npo_solve_adj(npo_plan plan, void* ws, const void* y, void* out, void* stream);

/* One predictor-corrector step u^n -> u^{n+1} at t_n = t0 + n dt (Sec. 2.3):
 * w_0 = S(E u^n + N(u^n)), w_c = S(E u^n + (N(u^n) + N(w_{c-1}))/2), c = 1..ncorr.
 * u_n and u_np1 may alias. */
npo_status npo_forward_step(npo_plan plan, void* ws, const void* u_n, void* u_np1, int64_t n,
                            void* stream);
/* The same step for callers that cannot allocate device memory (code under
 * HIP stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * instead of a caller workspace it uses a fixed device array of
 * NPO_SCRATCH_BYTES that the library holds on every device it runs on until
 * the process ends.  Results are bitwise those of npo_forward_step.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * Grids whose workspace_bytes exceed NPO_SCRATCH_BYTES are rejected with
 * NPO_EINVAL before anything is enqueued; the current device must be the
 * plan's.  Every call on one device shares that device's array: calls that
 * overlap on one device (several streams or threads) race and must be
 * serialised by the caller.  u_n and u_np1 may alias. */
#define NPO_SCRATCH_BYTES (64ll << 20)
npo_status npo_forward_step_noalloc(npo_plan plan, const void* u_n, void* u_np1, int64_t n, void* stream);
/* Exact discrete adjoint of that step (W inner product): lam_n = Phi'(u_n)^dag lam_np1
 * (Sec. 2 adjoint equations, integrated backward). lam_n may alias lam_np1. */
npo_status npo_adjoint_step(npo_plan plan, void* ws, const void* u_n, const void* lam_np1,
                            void* lam_n, int64_t n, void* stream);

/* The continuous adjoint (Sec. 2: the adjoint momentum and continuity
 * equations with the zero adjoint flux, integrated backwards from the
 * compatibility condition), discretised with the direct stepper of Sec. 2.3
 * rather than transposing it.  Its convective term, in rotational form with
 * V = U e_z + u and Omega = curl V, is
 *   Nc(u; y) = P_K F[Omega x Y] + curl P_K F[Y x V]
 * (the adjoint term -(V.grad) y + (grad V)^T y of the paper up to a gradient
 * and the sign of the backward time), and the backward step from t_{n+1} to
 * t_n is
 *   v_0 = S(E lam + Nc(u^{n+1}; lam)),  v_c = S(E lam + (Nc(u^{n+1}; lam) + Nc(u^n; v_{c-1}))/2),
 *   lam^n = v_ncorr,
 * the first term at t_{n+1}, the second at t_n.  Its gradient differs from the
 * exact discrete one by the discretisation error.
 *   npo_nonlinear_adj_cont: out = Nc(u; y) at time t;
 *   npo_adjoint_step_cont:  lam_n from lam_np1 with the direct fields u_n and
 *                           u_np1 (lam_n may alias lam_np1);
 *   npo_plan_set_adjoint:   kind 0 (default) makes the adjoint sweeps
 *                           (npo_adjoint_run, its hybrid form, npo_iterate)
 *                           use the exact discrete adjoint, kind 1 the
 *                           continuous one; the continuous sweeps make u^{n+1}
 *                           of each segment's last step with one forward step
 *                           (not counted in n_recompute) and keep it in the
 *                           workspace, and replay captured graphs for the
 *                           forward advances only.  Batches (npo_batch_*) take the
 *                           discrete adjoint only: NPO_EUNSUPPORTED otherwise. */
npo_status npo_nonlinear_adj_cont(npo_plan plan, void* ws, const void* u, double t, const void* y, void* out,
                                  void* stream);
npo_status npo_adjoint_step_cont(npo_plan plan, void* ws, const void* u_n, const void* u_np1,
                                 const void* lam_np1, void* lam_n, int64_t n, void* stream);
npo_status npo_plan_set_adjoint(npo_plan plan, int32_t kind);

/* Forward sweep over the plan's nsteps from u0 to uN, storing binomial
 * checkpoints (Sec. 2.4) into `ckpt`, an arena of n_ckpt fields (n_ckpt >= 1;
 * slot 0 receives u0).  The arena must not be touched before the matching
 * npo_adjoint_run. */
npo_status npo_forward_run(npo_plan plan, void* ws, void* ckpt, int32_t n_ckpt, const void* u0,
                           void* uN, void* stream);
/* The same sweep recording energy diagnostics (the growth decompositions
 * G = E/E0, G_z = E_z/E0, G_rtheta = (E_r + E_theta)/E0 of Sec. 3-4, and the
 * relative energy in the highest azimuthal and axial modes of the resolution
 * criterion of Sec. 2.3) as it goes: row n / stride of hist_dev (device,
 * 5 doubles a row, layout of npo_energy_diag) receives those of u^n for
 * n = 0, stride, 2 stride, ... < nsteps, and row (nsteps - 1) / stride + 1 those
 * of u^N, so hist_dev holds (nsteps - 1) / stride + 2 rows.  The checkpoints
 * and uN are those of npo_forward_run. */
npo_status npo_forward_run_diag(npo_plan plan, void* ws, void* ckpt, int32_t n_ckpt, const void* u0, void* uN,
                                double* hist_dev, int32_t stride, void* stream);
/* Backward adjoint sweep from lamN to lam0 using the checkpoints of the last
 * npo_forward_run with the same arena and n_ckpt.  *n_recompute (host) receives
 * the forward steps re-advanced from checkpoints; together with the nsteps-1
 * advances of the forward sweep they equal S N - beta(N_G+1, S-1) (Sec. 2.4).
 * The result does not depend on n_ckpt. */
npo_status npo_adjoint_run(npo_plan plan, void* ws, void* ckpt, int32_t n_ckpt, const void* lamN,
                           void* lam0, int64_t* n_recompute, void* stream);
/* Host-side count of the checkpoint schedule without running it. */
npo_status npo_ckpt_count(int64_t nsteps, int32_t n_ckpt, int64_t* n_recompute);

/* Two-level checkpointing (Sec. 2.4, memory checkpoints combined with a slower
 * tier; here pinned host memory stands in for the paper's disc files).  The
 * horizon is cut into n_file + 1 equispaced intervals (interval i covers steps
 * floor(i N / (n_file+1)) .. floor((i+1) N / (n_file+1)) - 1).
 * npo_forward_run_hybrid stores the start state of every interval but the last
 * in host_tier (caller-owned pinned host memory, hipHostMalloc, n_file fields
 * of field_bytes) and advances those intervals without device checkpoints; the
 * last interval is swept with the binomial device checkpoints of
 * npo_forward_run (arena of n_ckpt fields).  npo_adjoint_run_hybrid reverses
 * the last interval from those checkpoints, then for each earlier interval
 * restores its start state from the host tier, re-advances it to place the
 * device checkpoints and reverses it.  *n_recompute receives all forward
 * advances of the adjoint sweep.  The gradient is bitwise that of
 * npo_forward_run / npo_adjoint_run.  n_file = 0 is the device-only schedule. */
npo_status npo_forward_run_hybrid(npo_plan plan, void* ws, void* ckpt, int32_t n_ckpt, void* host_tier,
                                  int32_t n_file, const void* u0, void* uN, void* stream);
npo_status npo_adjoint_run_hybrid(npo_plan plan, void* ws, void* ckpt, int32_t n_ckpt, const void* host_tier,
                                  int32_t n_file, const void* lamN, void* lam0, int64_t* n_recompute,
                                  void* stream);
/* Forward advances of the hybrid adjoint sweep for n_file host checkpoints
 * (host arithmetic only): for equal intervals of length l this is the paper's
 * (N_F + 1) N_rec - N_init with N_rec the advances to recover an interval from
 * n_ckpt memory checkpoints and N_init = l - 1 (the last interval's checkpoints
 * are placed by the initial forward sweep). */
npo_status npo_hybrid_count(int64_t nsteps, int32_t n_ckpt, int32_t n_file, int64_t* n_recompute);
/* The number of host checkpoints n_file in [0, max_file] minimising the
 * recovery time of Sec. 2.4, T = n_file t_io + advances(n_file) t_step, with
 * t_io the time to restore one field from the host tier and t_step that of one
 * forward step (both measured by the caller); *t_rec (optional) receives T. */
npo_status npo_hybrid_plan(int64_t nsteps, int32_t n_ckpt, double t_io, double t_step, int32_t max_file,
                           int32_t* n_file, double* t_rec);

/* Energy diagnostics of a field u (deterministic fixed-order reductions):
 * out_dev[0..2] = E_r, E_theta, E_z (E_c = <u_c, u_c>_W / 2, their sum is E(u)),
 * out_dev[3] = energy in the modes m = M, out_dev[4] = energy in the modes
 * |k| = K (divided by E0 these are the paper's resolution measures e_M, e_K of
 * Sec. 2.3, read as energy fractions).  spec_dev (optional, device,
 * (M+1)(2K+1) doubles, [m][kk] in the field's axial order) receives the energy
 * of every stored mode (for m = 0 the modes +k and -k separately, as in
 * <.,.>_W).  ws: workspace of workspace_bytes (reduction partials). */
npo_status npo_energy_diag(npo_plan plan, void* ws, const void* u, double* out_dev, double* spec_dev,
                           void* stream);
/* out_dev[0] = <a,b>_W (deterministic fixed-order reduction). */
npo_status npo_inner(npo_plan plan, void* ws, const void* a, const void* b, double* out_dev,
                     void* stream);
/* out = P_h u: W-orthogonal projection onto admissible perturbations (zero
 * wall velocity, zero discrete divergence at every node, zero flux and u_r = 0
 * for the mean mode); the normal equations are solved twice (one refinement).
 * out may alias u. */
npo_status npo_project(npo_plan plan, void* ws, const void* u, void* out, void* stream);
/* Gradient step of Sec. 2.2 with every scalar computed and kept on the device:
 * g is the projected W-gradient of the gain (udag = -g, the paper's sign
 * convention u_dag(T) = -u(T)).  On `stream` the call forms
 *   E0dag = <g,g>_W / 2,  C0 = <u0, udag>_W,
 *   alpha_max = (E0dag/e0 - C0^2/(4 e0^2))^(-1/2)   (infinite if g || u0),
 *   lambda_+  = '+' root of the energy constraint at step al (discriminant
 *               clamped at 0, where it sits at al = alpha_max),
 *   u_new     = (1 + lambda_+ al) u0 - al udag, rescaled to energy e0,
 * with al = alpha if alpha > 0, else al = alpha_max (an empty step when that is
 * infinite).  info_dev (device, 5 doubles) receives E0dag, C0, alpha_max,
 * lambda_+ and E_new, the energy of u_new before the final rescale (equal to
 * e0 up to rounding when lambda_+ is exact).  u_new must not alias u0 or g.
 * ws: workspace of workspace_bytes (reduction partials). */
npo_status npo_update(npo_plan plan, void* ws, const void* u0, const void* g, double e0,
                      double alpha, void* u_new, double* info_dev, void* stream);

/* One adjoint-looping iteration (Sec. 2.1-2.2) on the host: requires that the
 * arena holds the forward sweep of u0 (npo_forward_run, or the accepted trial
 * of the previous iterate) with u^N in uN.  Runs the adjoint sweep, projects
 * the gradient, and does the backtracking line search (alpha = alpha_max,
 * halve while G does not increase, stop when |dG/G| < tol or after
 * max_halvings).  On acceptance u0 and uN hold the new iterate and the arena its
 * sweep.  stats (host, 8 doubles): G_old, G_new, alpha, alpha_max, E0dag, C0,
 * accepted (1/0), forward sweeps run.  A non-finite G_old, E0dag or C0 (a state
 * that has blown up) ends the call at once with NPO_OK, accepted = 0, G_new =
 * G_old and nothing changed, so that the caller sees the non-finite gain.
 * Synchronises the stream. */
npo_status npo_iterate(npo_plan plan, void* ws, void* ckpt, int32_t n_ckpt, void* u0, void* uN,
                       double e0, double tol, int32_t max_halvings, double* stats, void* stream);

/* Launch shapes of the transform kernels (the autotuner's knobs): zgroup =
 * fields per axial-transform block (1..3), zb_fwd / zb_adj = axial points per
 * azimuthal-transform block in the forward / adjoint products (2, 4 or 8,
 * dividing nz); zb_fwd or zb_adj = -L selects the wave-resident azimuthal
 * kernels with L lanes per axial column (sequences in registers, cross-lane
 * radix-2 stages): L = 8 for ntheta in {24, 48, 96} and nz a multiple of 8,
 * L = 16 for ntheta in {48, 96} and nz a multiple of 4.  Shapes whose LDS tiles exceed 160 KiB are rejected
 * (NPO_EINVAL).  Results do not depend on the shapes. */
npo_status npo_plan_set_tuning(npo_plan plan, int32_t zgroup, int32_t zb_fwd, int32_t zb_adj);
npo_status npo_plan_get_tuning(npo_plan plan, int32_t* zgroup, int32_t* zb_fwd, int32_t* zb_adj);

/* Launch shape of the radial kernels (the per-mode solves of Sec. 2.3 and
 * their transposes, the autotuner's other knob): rg = axial wavenumbers |k|
 * per block (4, 8 or 16; a block holds the +k and -k modes of rg wavenumbers
 * at one azimuthal index, 32 rg threads).  Larger blocks read longer runs of
 * each radial row, smaller ones give small grids more blocks.  Any other value
 * is NPO_EINVAL.  Results do not depend on rg.  Default 16. */
npo_status npo_plan_set_radial_block(npo_plan plan, int32_t rg);
npo_status npo_plan_get_radial_block(npo_plan plan, int32_t* rg);

/* Step graphs for the checkpointed sweeps (enable = 1): npo_forward_run and
 * npo_adjoint_run (and so npo_iterate) replay one captured HIP graph per
 * forward advance and per adjoint step (Sec. 2.3 step, Sec. 2.4 sweeps)
 * instead of launching each step's kernels; the step index the time depends on
 * is read from the workspace.  Graphs are captured on first use for a
 * workspace (a new workspace, new launch shapes or enable = 0 drop them) and
 * are not used while the sampling profiler runs.  Results are bitwise those of
 * enable = 0.  Default 0. */
npo_status npo_plan_set_graphs(npo_plan plan, int32_t enable);

/* CFL monitor (enable = 1): every forward step folds the CFL number of its
 * state u^n, max over the physical 3/2-rule points of
 * dt (|u_z + U| / dz + |u_theta| / (r dtheta) + |u_r| / dr_j) with dr_j the
 * smaller gap to a neighbouring radial node (2 r_0 at the first node), into a
 * device maximum kept in the workspace (the explicit convective terms of the
 * predictor-corrector step are stable only below a bound of order one).
 * Supported by the LDS-staged azimuthal kernels of every length (tuning
 * zb_fwd > 0); with the wave-resident kernels (zb_fwd < 0) the monitor reads
 * 0.  Drops captured graphs.  npo_cfl_read copies the maximum so far into out_dev (one
 * device double) on `stream` and, with reset = 1, clears it; the maximum lives
 * in the workspace, so clear it (a read with reset = 1) before the first
 * monitored step of a new workspace. */
npo_status npo_plan_set_cfl_monitor(npo_plan plan, int32_t enable);
npo_status npo_cfl_read(npo_plan plan, void* ws, double* out_dev, int32_t reset, void* stream);

/* Failure injection for tests of error handling (no device fault is made):
 * after `after` more calls of the step driver at `site` (1: forward step,
 * 2: adjoint step; 0: off), the next call returns NPO_EHIP from the entry point
 * that made it, as a failed launch would, before enqueueing that step.  Steps
 * replayed from captured graphs are not counted. */
npo_status npo_plan_inject_fault(npo_plan plan, int32_t site, int64_t after);

/* out = scale * q (.) lam with q = 2 pi L_z c_m w_j: converts the W-gradient
 * lam of a real functional into the gradient with respect to the real and
 * imaginary parts of the stored coefficients (m = 0 entries at +k and -k count
 * as independent coordinates).  out may alias lam. */
npo_status npo_euclid_grad(npo_plan plan, const void* lam, double scale, void* out, void* stream);

/* u *= sqrt(e0 / E(u)), E(u) = <u,u>_W / 2, on the device. */
npo_status npo_normalize(npo_plan plan, void* ws, void* u, double e0, void* stream);

/* Batched instances (many optimisation instances of uneven grid and parameter
 * sizes advanced together).  A batch groups its plans into shape classes
 * (equal nr, ntheta, nz, corrector passes, launch shapes and device); a
 * batched step issues each kernel of the step once per class for all of the
 * class's instances, every block reading its instance's plan constants,
 * buffers and evaluation time from a device work-descriptor table (built on
 * the first step with a given set of workspaces and kept by the batch); a
 * class whose kernels have no batched form (transform lengths without the
 * pruned compiled kernels, the wave-resident azimuthal kernels) runs its
 * instances' steps one after another instead.  The plans must share nsteps,
 * and stay owned by the caller until npo_batch_destroy.  Results are bitwise
 * those of the instances' own calls. */
typedef struct npo_batch_s* npo_batch;
npo_status npo_batch_create(const npo_plan* plans, int32_t n, npo_batch* out);
npo_status npo_batch_destroy(npo_batch batch);
/* Shape classes, instances advanced by batched launches, and kernel launches
 * of the last batched step (independent of the instance count for batched
 * classes). */
npo_status npo_batch_info(npo_batch batch, int32_t* n_classes, int32_t* n_batched, int32_t* launches);
/* Every instance's device step index (the evaluation time t0 + n dt of its
 * next step) set to n. */
npo_status npo_batch_set_steps(npo_batch batch, void* const* ws, int64_t n, void* stream);
/* One step of every instance (Sec. 2.3 step, or its exact adjoint):
 * phase 0: states[i] <- Phi(states[i]) at each instance's step index, which
 * then increases by one; phase 1: states[2i+1] <- Phi'(states[2i])^dag
 * states[2i+1] at the step index, which then decreases by one.  ws[i] is
 * instance i's workspace (its `cur` and `lam` fields carry the states during
 * the step). */
npo_status npo_batch_step(npo_batch batch, void* const* states, void* const* ws, int32_t phase, void* stream);
/* Checkpointed forward and adjoint sweeps of every instance in lockstep (one
 * binomial schedule, Sec. 2.4, for the shared nsteps and n_ckpt; advances and
 * adjoint steps are batched steps replayed from one captured graph per phase),
 * with the contracts of npo_forward_run / npo_adjoint_run per instance:
 * ckpt[i] an arena of n_ckpt fields of instance i. */
npo_status npo_batch_forward_run(npo_batch batch, void* const* ws, void* const* ckpt, int32_t n_ckpt,
                                 void* const* u0, void* const* uN, void* stream);
npo_status npo_batch_adjoint_run(npo_batch batch, void* const* ws, void* const* ckpt, int32_t n_ckpt,
                                 void* const* lamN, void* const* lam0, int64_t* n_recompute, void* stream);

/* Sampling profiler: from npo_profile_begin until npo_profile_read, every
 * stride-th launch of each kernel family is bracketed by HIP events recorded
 * on the stream it is launched on.  npo_profile_read (host arrays of
 * NPO_KERNEL_FAMILIES entries) synchronises on the recorded events and returns
 * launch counts, sampled counts and the mean sampled duration in ms.
 * Families: 0 curl, 1-3 forward axial-inverse / azimuthal / axial-forward
 * transforms, 4-6 the same for the adjoint, 7 predictor solve, 8 corrector
 * solve, 9 plain solve, 10 adjoint solve, 11 adjoint combine, 12 reduction,
 * 13 projection, 14 axpby, 15 adjoint solve of the composed input, 16 adjoint
 * axial-inverse transform of the adjoint field alone (when the forward
 * transforms of the same state are reused). */
#define NPO_KERNEL_FAMILIES 17
npo_status npo_profile_begin(npo_plan plan, int32_t stride);
npo_status npo_profile_read(npo_plan plan, int64_t* launches, int64_t* sampled, double* avg_ms);

#ifdef __cplusplus
}
#endif
#endif /* NPO_H */
