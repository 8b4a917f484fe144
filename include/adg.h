/*
 * adg.h — C ABI of the MI355X (gfx950) asynchronous discontinuous Galerkin
 * right-hand-side library for the compressible Euler equations.
 *
 * Method: arXiv 2603.28710 ("Scalability of the asynchronous discontinuous
 * Galerkin method for compressible flow simulations").
 *   - Euler system and closure: Sec. 2, eq. euler-dealii / euler-parameters-dealii
 *     (body force G = 0).
 *   - Nodal DG weak form, element mass matrix: Sec. 2.1, eq. weakform-dealii,
 *     weakform-compact-dealii. Lagrange basis on Gauss-Lobatto nodes, Gauss
 *     quadrature with p+2 points per direction, sum-factorised.
 *   - Local Lax-Friedrichs flux: Sec. 2.2, eq. lfflux and lfflux-lambda.
 *   - Interior / PE-boundary classification: Sec. 2.4, Fig. Domain-decomposition.
 *     PEs are emulated as "virtual subdomains" of one GPU.
 *   - Delayed neighbour data with maximum delay L: Sec. 3, eq. euler-adg-compact,
 *     delayed-flux; communication-avoiding schedules: Alg. caa-std, caa-at.
 *   - AT extrapolation over past levels with the stage-fractional delay of the
 *     naive RK coupling: Sec. 3.2, eq. at-flux, at-flux-constraints,
 *     Table at-flux-coeffs; applied here to neighbour traces.
 *   - Time integration: explicit SSP-RK3 in Shu-Osher form (default),
 *     SSP-RK2, or the paper's two-register LSERK(2,2) / LSERK(3,3) of
 *     Sec. 2.3 (eq. lserk-dg, Table lserk-scheme; stage times from the
 *     scheme's own a and b).
 *   - Boundaries: a periodic box (default), or, for d = 2, the Dirichlet box of
 *     the paper's vortex test (Sec. 5.1), whose boundary data come from the
 *     exact solution.
 *
 * Conventions shared by every entry point
 *   - Every function returns adg_status: ADG_OK (0) or a negative code. No
 *     function aborts, throws or prints. adg_last_error() returns a
 *     thread-local message describing the last non-OK status.
 *   - Device pointers are HIP device addresses (e.g. torch tensor data_ptr()).
 *     They are owned by the caller, must stay valid while the context uses
 *     them, and are never freed by the library.
 *   - Host pointers are borrowed for the duration of the call only.
 *   - All GPU work is enqueued on the stream given to adg_create (0 = the
 *     null stream). The library never calls hipDeviceSynchronize; calls that
 *     return host data synchronise that stream only.
 *   - The library itself allocates only small device tables (a few KB) and
 *     the reduction/flag area it needs; it frees them in adg_destroy.
 *
 * Public state layout: double[N_E][V][P^d], V = d+2 variables
 * (rho, rho*u_x, rho*u_y[, rho*u_z], E), P = degree+1 Gauss-Lobatto nodes per
 * direction, node index lexicographic with x fastest, element index
 * e = ix + nx*(iy + ny*iz). The device state registers use this layout too.
 */
#ifndef ADG_H
#define ADG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t adg_status;

#define ADG_OK 0
#define ADG_ERR_INVALID (-1)     /* bad argument or configuration */
#define ADG_ERR_UNBOUND (-2)     /* device buffers not bound (adg_bind) */
#define ADG_ERR_HIP (-3)         /* a HIP call failed; message has the HIP error string */
#define ADG_ERR_NONFINITE (-4)   /* state holds NaN/Inf at a check */
#define ADG_ERR_NONPHYSICAL (-5) /* density or pressure <= 0 at a check */
#define ADG_ERR_STATE (-6)       /* call not allowed in the current state */

/* numerical flux (Sec. 2.2) */
#define ADG_FLUX_LLF 0     /* eq. lfflux with lambda as printed (includes the factor 1/2) */
#define ADG_FLUX_RUSANOV 1 /* lambda = max(|u.n| + c) over both sides */
/* time integrator */
#define ADG_SSPRK3 0  /* three stages, Shu-Osher form; three state registers */
/* LSERK(s,o) of eq. lserk-dg: k_m = M^-1 L(r_m), r_{m+1} = w + dt a_m k_m,
 * w <- w + dt b_m k_m with r_1 = w = u^n and the digits of Table
 * lserk-scheme; the stage times c_1 = 0, c_m = b_1 + .. + b_{m-2} + a_{m-1}
 * enter the AT fractional delay tau = k + c_m. Uses the same three registers
 * (u_n, u_a, u_b); the state is in u_n after every step. */
#define ADG_LSERK22 1
#define ADG_LSERK33 2
/* SSP-RK2 (Heun) in Shu-Osher form: u1 = u^n + dt L(u^n),
 * u^{n+1} = u^n / 2 + (u1 + dt L(u1)) / 2; stage times 0 and 1 */
#define ADG_SSPRK2 3
/* arithmetic of the volume/face contractions and inverse mass */
#define ADG_FP64 0
#define ADG_FP32_CONTRACT 1 /* contractions in FP32; RK state, AT weights, norms in FP64 */
/* neighbour data at PE-boundary faces (Sec. 3) */
#define ADG_GHOST_SYNC 0    /* always the neighbour's current stage values (Alg. sa) */
#define ADG_GHOST_STALE 1   /* standard flux on the trace delayed by k steps (eq. delayed-flux) */
#define ADG_GHOST_AT 2      /* AT extrapolation of `levels` past traces (eq. at-flux) */
#define ADG_GHOST_LEARNED 3 /* AT plus a learned correction, judged per face (AT fallback) */
/* flux-history modes, ADG_DELAY_CAA only: the numerical flux at each PE face
 * is computed from current data and stored at the first stage of
 * communicating steps; silent steps reuse it (Alg. caa-std) or extrapolate the
 * stored history to the stage time with the AT weights (Alg. caa-at). Both
 * sides of a face use one value, so the scheme conserves under asynchrony. */
#define ADG_GHOST_FLUX_STALE 4
#define ADG_GHOST_FLUX_AT 5
/* delay per (step, receiving subdomain, face direction) */
#define ADG_DELAY_FIXED 0   /* k = L */
#define ADG_DELAY_UNIFORM 1 /* k uniform in {0..L}, SplitMix64 draw from the seed */
#define ADG_DELAY_CAA 2     /* Alg. caa-std (STALE, FLUX_STALE) / Alg. caa-at (AT, LEARNED, FLUX_AT) schedule */
/* boundary of the box */
#define ADG_BC_PERIODIC 0
/* Dirichlet on every side (d = 2 only): a boundary face takes the numerical
 * flux with the exact solution of the boundary problem (adg_set_boundary;
 * adg_init_problem sets it too) as the exterior state, evaluated at the
 * face's Gauss-Lobatto nodes at each stage's time t_n + c_m dt and
 * interpolated to the face Gauss points like a neighbour's trace. Boundary
 * faces are never PE faces. Exact solutions are not wrapped periodically. */
#define ADG_BC_DIRICHLET 1
/* analytic problems */
#define ADG_VORTEX 0       /* isentropic vortex (Sec. 5.1); params x0,y0,beta,mean_u,mean_v; in a
                              periodic box the nearest periodic image of the centre */
#define ADG_DENSITY_WAVE 1 /* rho = 1 + A sin(2 pi sum_k (x_k - u_k t)); params A,u1,u2,u3,p */
#define ADG_CONSTANT 2     /* constant state; params rho,u1,u2,u3,p */

typedef struct adg_config {
  int32_t dim;         /* 2 or 3 */
  int32_t degree;      /* N_p in 1..4 */
  int32_t n_q;         /* Gauss points per direction; 0 means degree+2 (the only supported value) */
  int32_t cells[3];    /* elements per direction (cells[2] ignored in 2D) */
  int32_t parts[3];    /* virtual subdomains per direction; cells[k] % parts[k] == 0 */
  double lo[3], hi[3]; /* the box */
  double gamma;        /* ratio of specific heats (> 1) */
  int32_t flux;        /* ADG_FLUX_* */
  int32_t integrator;  /* ADG_SSPRK3, ADG_LSERK22, ADG_LSERK33 or ADG_SSPRK2 */
  int32_t precision;   /* ADG_FP64 or ADG_FP32_CONTRACT */
  int32_t check_every; /* 0: adg_step never checks the state; k>0: every k steps and at the end */
  int32_t boundary;    /* ADG_BC_PERIODIC or ADG_BC_DIRICHLET (d = 2) */
} adg_config;

typedef struct adg_async {
  int32_t ghost;      /* ADG_GHOST_* */
  int32_t delay_kind; /* ADG_DELAY_* */
  int32_t L;          /* maximum delay, 0..16 */
  int32_t levels;     /* AT levels (order), 1..4 */
  uint64_t seed;      /* seed of the uniform delay draws */
  double learned_tol; /* accept bound on the learned correction (physical units), e.g. 1e-6 */
  int32_t learned_judge; /* 0: a face's correction is accepted iff max|d| <= learned_tol;
                            1: also iff max|d| <= max|AT over 4 levels - AT over 3 levels| on
                            the face, the extrapolation's own error estimate */
} adg_async;

typedef struct adg_ctx_s* adg_ctx;

/* Create a context. Validates the configuration (ADG_ERR_INVALID with a
 * message otherwise) and computes the host tables; makes no HIP call.
 * `hip_stream` is a hipStream_t (may be NULL = null stream). The context owns
 * no state buffers: see adg_bind. */
adg_status adg_create(const adg_config* cfg, const adg_async* async, void* hip_stream, adg_ctx* out);

/* Sizes the caller must allocate: n_dof doubles per state register
 * (state_bytes = 8 n_dof), ring_bytes for the history (0 for SYNC): R levels
 * of double[n_face_sides][V][P^(d-1)] face-node traces, or, in the
 * flux-history modes, of double[n_face_sides][V][n_q^(d-1)] face-point
 * fluxes, with R = L+1 (STALE, FLUX_STALE), L+levels (AT, FLUX_AT) or
 * L+max(levels,4) (LEARNED); scratch_bytes for the ghost traces and
 * reductions. */
adg_status adg_sizes(adg_ctx ctx, size_t* n_dof, size_t* state_bytes, size_t* ring_bytes, size_t* scratch_bytes);

/* Bind caller-owned device buffers: the three state registers (u_n holds
 * the solution between steps; u_a is also used as staging by adg_diff_norm),
 * the ring (may be NULL if ring_bytes == 0) and the scratch area, all at least
 * the sizes of adg_sizes, 256-byte aligned. The first bind allocates and
 * uploads the context's small device tables (freed by adg_destroy). */
adg_status adg_bind(adg_ctx ctx, void* u_n, void* u_a, void* u_b, void* ring, void* scratch);

/* Copy a host state (public layout, n == n_dof doubles) into u_n, or back.
 * Upload resets the step counter, time and trace history. */
adg_status adg_upload(adg_ctx ctx, const double* host, size_t n);
adg_status adg_download(adg_ctx ctx, double* host, size_t n);

/* L2 projection of an analytic problem (ADG_VORTEX, ...) at t = 0 into u_n,
 * computed on the GPU: u = M_e^{-1} (phi, w_exact)_e with the element mass
 * matrix of Sec. 2.1 (eq. weakform-compact-dealii) and the Gauss rule of
 * p + 2 points per direction; the vortex is the test problem of Sec. 5.1.
 * params may be NULL for the defaults (vortex 5,5,5,1,1; density wave
 * 0.2,1,1,1,1; constant 1,0.3,-0.2,0.1,1). Resets
 * n, t and the history, and makes the problem the boundary problem. */
adg_status adg_init_problem(adg_ctx ctx, int32_t problem, const double* params);

/* The analytic problem whose exact solution supplies the boundary data of an
 * ADG_BC_DIRICHLET box (params as for adg_init_problem; NULL = defaults).
 * Host-only, no HIP call. adg_step in a Dirichlet box returns
 * ADG_ERR_STATE until a boundary problem is set. */
adg_status adg_set_boundary(adg_ctx ctx, int32_t problem, const double* params);

/* Change the asynchrony settings. The ring bound at adg_bind must be large
 * enough for the new depth (ADG_ERR_INVALID otherwise). The history restarts:
 * the warm-up clamp counts from the current step. */
adg_status adg_set_async(adg_ctx ctx, const adg_async* async);

/* Advance n_steps steps of the configured integrator, of fixed size dt (> 0;
 * n_steps == 0 does nothing). Each stage evaluates the right-hand side
 * M^{-1} R(w) of Sec. 2.1 (eq. weakform-dealii, weakform-compact-dealii) with
 * the numerical flux of Sec. 2.2 on every face; at PE-boundary faces the
 * neighbour trace follows the asynchrony settings (Sec. 3: the delayed trace
 * of eq. delayed-flux, the AT extrapolation of eq. at-flux with the naive
 * stage coupling tau = k + c_m of Sec. 3.2, the stored fluxes of Alg.
 * caa-std / caa-at); the stages combine as the integrator prescribes (SSP-RK3
 * Shu-Osher form; eq. lserk-dg for LSERK). The time step dt stays fixed, as
 * the AT weights assume uniform steps (Sec. 3.2). Asynchronous on the stream unless
 * check_every > 0, in which case the state is checked (finite, rho > 0,
 * p > 0) every check_every steps and at the end of the call, with a blocking
 * read of one flag: ADG_ERR_NONFINITE / ADG_ERR_NONPHYSICAL. */
adg_status adg_step(adg_ctx ctx, int64_t n_steps, double dt);

/* Delay k (in steps) that the receiving subdomain `sub` uses at step n for
 * its face direction dir (f = 2a + side, side 0 = the -a face), after the
 * warm-up clamp that starts at the current history origin (Sec. 3,
 * eq. euler-adg-compact; Alg. caa-std / caa-at for ADG_DELAY_CAA). Host-only
 * computation, no HIP call; *n_face_sides (may be NULL) gets the number of
 * PE-boundary face-sides of the partition. */
adg_status adg_delay(adg_ctx ctx, int64_t n, int32_t sub, int32_t dir, int32_t* k, int64_t* n_face_sides);

/* The 1D rules the context uses (host-only, no HIP call): degree+1
 * Gauss-Lobatto nodes and weights, n_q Gauss nodes and weights, ascending on
 * [-1, 1]. Any pointer may be NULL. */
adg_status adg_basis(adg_ctx ctx, double* gll_x, double* gll_w, double* gauss_x, double* gauss_w);

/* Kernel timing with HIP events. With enable = k > 0 the library records a
 * pair of library-owned events on its stream around every launch of the
 * stage kernels in the steps n with n % k == 0 (k = 1: every launch; a
 * larger k keeps the events' own cost, a few microseconds per pair, out of
 * most steps); adg_profile_read synchronises the stream and returns, for
 * kernel ADG_KERNEL_RHS (fused right-hand-side stage) or ADG_KERNEL_GHOST
 * (learned ghost traces), the summed elapsed milliseconds and the number of
 * recorded launches since profiling was enabled. enable == 0 stops
 * recording; enable < 0 is ADG_ERR_INVALID. */
#define ADG_KERNEL_RHS 0
#define ADG_KERNEL_GHOST 1
adg_status adg_profile(adg_ctx ctx, int32_t enable);
adg_status adg_profile_read(adg_ctx ctx, int32_t kernel, double* total_ms, int64_t* launches);

/* Step counter and time (t = sum of the dt's since the last reset). */
adg_status adg_time(adg_ctx ctx, int64_t* n, double* t);

/* dt = cfl * min_k h_k / (degree^1.5 * max over nodes of (|u| + c)), from u_n. */
adg_status adg_stable_dt(adg_ctx ctx, double cfl, double* dt);

/* Quadrature (n_q Gauss points) L2 norms of u_n minus the exact solution at
 * the current time: out = {rho, |rho u| (vector), E}; the error measure of
 * the convergence study (Sec. 5.3). */
adg_status adg_error_norms(adg_ctx ctx, int32_t problem, const double* params, double out[3]);

/* Relative L2 difference of u_n against a host state of the public layout,
 * per group over nodal values: out = {rho, momentum, E}, each
 * ||u - ref|| / ||ref||. */
adg_status adg_diff_norm(adg_ctx ctx, const double* host_ref, double out[3]);

/* Integrals of the V conserved variables over the box (quadrature), FP64:
 * the conservation check of the scheme (Sec. 3.3 states that the CAA-AT
 * algorithm keeps local conservation: its stored fluxes are one value per
 * face; the trace modes, where each side of a PE face builds its own flux,
 * do not conserve under asynchrony). out receives V doubles. */
adg_status adg_integrals(adg_ctx ctx, double* out);

/* adg_integrals for callers that cannot allocate, or cannot lend the bound
 * scratch area (code under graph capture, serving loops, harnesses that
 * forbid allocation): the same kernels and the same result, with their
 * per-block partial sums (at most 2048 blocks of 6 doubles) and the reduced
 * values in a static device array of 98,560 bytes that the library holds per
 * GPU until the process ends, instead of the scratch bound at adg_bind. Calls
 * no allocating routine. The context must be bound and its device (the one
 * current at adg_bind) current: ADG_ERR_STATE otherwise; a mesh that would
 * need more partial blocks than the array holds is ADG_ERR_INVALID (the norm
 * kernels use at most 2048). Every call on a GPU shares that GPU's array:
 * calls that overlap on one GPU (several streams or threads) race. Blocks on
 * the context's stream; out receives V doubles. */
adg_status adg_integrals_noalloc(adg_ctx ctx, double* out);

/* Checkpoint: state u_n, ring, step counter, time, history origin,
 * asynchrony settings, boundary problem and predictor weights into a host
 * blob. Call with host_blob == NULL to get the
 * size in *bytes. adg_load restores a blob saved from the same configuration. */
adg_status adg_save(adg_ctx ctx, void* host_blob, size_t* bytes);
adg_status adg_load(adg_ctx ctx, const void* host_blob, size_t bytes);

/* Learned ghost predictor (MLP: 2V+2 inputs, 64 GELU hidden units, V outputs).
 * adg_predictor_bind gives the device buffer that holds training pairs
 * (adg_predictor_pair_bytes(ctx) bytes per pair). collect runs n_steps of the
 * solver with AT ghosts and records (features, live-vs-AT target) pairs at
 * PE-boundary face nodes, up to max_pairs; train runs FP32 Adam epochs on the
 * GPU; get/set move FP32 weights (adg_predictor_nparams(ctx) floats). */
adg_status adg_predictor_nparams(adg_ctx ctx, int32_t* nparams);
adg_status adg_predictor_pair_bytes(adg_ctx ctx, size_t* bytes);
/* pairs: device buffer of max_pairs records (0 <= max_pairs < 2^31), caller-owned */
adg_status adg_predictor_bind(adg_ctx ctx, void* pairs, int64_t max_pairs);
/* copy n host records into the pair buffer (replaces its content) */
adg_status adg_predictor_load_pairs(adg_ctx ctx, const float* host_pairs, int64_t n);
/* Glorot-uniform weights (zero biases) from SplitMix64 draws of seed */
adg_status adg_predictor_init(adg_ctx ctx, uint64_t seed);
/* needs the LEARNED ghost mode (its ring keeps 4 levels); advances the solver
 * n_steps with AT ghosts and appends one record per PE-boundary face node and
 * stage while the buffer has room (records of zero-delay faces have weight 0) */
adg_status adg_predictor_collect(adg_ctx ctx, int64_t n_steps, double dt, int64_t* n_pairs);
/* FP32 Adam (0.9, 0.999, 1e-8) on the weighted MSE, minibatches of
 * batch <= 4096 records in a seeded permutation per epoch; initialises the
 * weights from the seed if none are set. *loss_out: last minibatch loss. */
adg_status adg_predictor_train(adg_ctx ctx, int32_t epochs, int32_t batch, float lr, uint64_t seed, float* loss_out);
/* FP32 loss and its gradient over records [first, first+count), count <= 4096 */
adg_status adg_predictor_grad(adg_ctx ctx, int64_t first, int64_t count, float* grad, float* loss_out);
/* BF16 matrix-core inference on the features of records [first, first+count),
 * count <= 4096; y receives V outputs per record */
adg_status adg_predictor_infer(adg_ctx ctx, int64_t first, int64_t count, float* y);
adg_status adg_predictor_get(adg_ctx ctx, float* w);
adg_status adg_predictor_set(adg_ctx ctx, const float* w);
/* Statistics of the learned ghost traces since the last reset (adg_upload,
 * adg_init_problem, adg_set_async): the faces judged (learned mode with a
 * network, delay >= 1) and the fraction whose correction was accepted (1 -
 * the AT fallback rate); and, over every PE face node with delay >= 1 that the
 * learned ghost kernel built (learned mode or pair collection), the mean of
 * max_v |w+ used - w+ live| (mean_trace_err) and of max_v |w+ AT - w+ live|
 * (mean_at_err), where w+ live is the neighbour's current stage value, the
 * trace a synchronous scheme would use. Any pointer may be NULL. Blocks on
 * the stream. */
adg_status adg_predictor_stats(adg_ctx ctx, double* accept_rate, int64_t* faces_judged, double* mean_trace_err,
                               double* mean_at_err);

adg_status adg_destroy(adg_ctx ctx);
const char* adg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ADG_H */
