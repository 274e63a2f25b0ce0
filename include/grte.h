/*
 * grte.h -- C ABI of the MI355X library for the asymptotic-preserving (AP)
 * time step of the 1-D gray radiative transfer equation
 *
 *   (1/c) d_t I + (1/eps) v d_x I = (sigma/eps^2)(a c T^4 - I),
 *   Cv d_t T = (sigma/eps^2)(rho - a c T^4),   rho = <I> = (1/2) int_{-1}^{1} I dv,
 *
 * ((1.1); sigma = sigma0 or sigma0 / T^3 as in (1.4)) with inflow data (4.1),
 * discretised with the even/odd parities (4.2) on the staggered grid
 * (4.3)-(4.4) and advanced by Algorithm 2 of Tang, Wang & Zhang,
 * arXiv 1811.05579 (prediction (4.5)/(5.2), correction (4.13) + (4.11)/(5.3),
 * projection (4.14)).
 *
 * Conventions
 *  - Every call returns a grte_status (0 = success, < 0 = error); no C++
 *    exception crosses the ABI.  On error nothing is partially committed
 *    unless stated.
 *  - N cells j = 0..N-1 on [0, L]; N+1 nodes i = 0..N (node i between cells
 *    i-1 and i).  P parity pairs p = 0..P-1 with mu_p > 0.
 *  - Parity arrays are cell-major, binary64: E[j*P + p] (cell centres,
 *    (4.3)) and O[i*P + p] (nodes, (4.4)); T[j] and sigma0[j] per cell.
 *  - The context owns all device memory.  Pointers passed in are borrowed for
 *    the duration of the call only; `on_device` != 0 means the pointer is
 *    device memory (copied on the context's stream), otherwise host memory.
 *  - All device work is ordered on the context's HIP stream (default: the
 *    null stream).  Calls that read results into host memory synchronise
 *    that stream; grte_step itself does not, unless `info` is non-NULL.
 *  - One context must not be used from two threads at once.
 */
#ifndef GRTE_H
#define GRTE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum grte_status {
    GRTE_OK = 0,
    GRTE_E_INVAL = -1,       /* NULL pointer, size or value out of range        */
    GRTE_E_NOMEM = -2,       /* device allocation failed                         */
    GRTE_E_HIP = -3,         /* a HIP runtime call or kernel launch failed       */
    GRTE_E_NOCONV = -4,      /* step completed, but the prediction iteration or
                                a Newton solve stopped at its cap (see info)    */
    GRTE_E_UNSUPPORTED = -5  /* size beyond the library's limits (N > 4096 or
                                P > 64)                                          */
} grte_status;

typedef struct grte_ctx grte_ctx;

/* Problem definition (fixed for the life of a context). */
typedef struct grte_problem {
    int nx;            /* number of cells N, 2 <= N <= 4096                      */
    int npairs;        /* parity pairs P = N_v / 2, 1 <= P <= 64                 */
    double length;     /* slab length L > 0                                      */
    double a;          /* radiation constant a > 0                               */
    double c;          /* speed of light c > 0                                   */
    double cv;         /* heat capacity Cv > 0                                   */
    int opacity_law;   /* m: 0 -> sigma = sigma0; 3 -> sigma = sigma0 / T^3 (1.4) */
} grte_problem;

/* Diagnostics of one step (filled only when a non-NULL pointer is passed). */
typedef struct grte_step_info {
    int pred_iters;       /* iterations of the prediction solve                 */
    int pred_converged;   /* 1 if the prediction met its tolerance              */
    int newton_max_iters; /* largest Newton iteration count over the cells      */
    int newton_failed;    /* cells whose Newton solve hit the cap               */
    int kstar_clamped;    /* sigma/T^3: cells with U* < 0 (K* taken as 0)       */
    int negative_root;    /* cells whose temperature equation has no root >= 0  */
    int sync_error;       /* 1 if a grid barrier of the prediction timed out
                             (the step's results are then invalid; GRTE_E_HIP) */
    int guess_accepted;   /* cells whose learned starting value already met the
                             residual bound (no Newton step taken)             */
    int guess_rejected;   /* cells whose learned start was unusable, had a
                             larger residual than T^n, or whose Newton from it
                             hit the cap: solved from T^n                      */
    int newton_total_iters; /* Newton iterations summed over the cells         */
    int guess_started;    /* cells whose Newton started from the learned value */
    int pred_floor_stop;  /* 1 if the prediction stopped at the rounding level
                             (counted in pred_converged; see grte_set_solver) */
    /* Energy balance of the step, (3.12)-(3.13): binary64 sums in a fixed
     * order (the same bits for the same state), formed by the projection
     * kernel on every step. */
    double energy_before;    /* E_tot^n = sum_j dx (rho^n_j / c + Cv T^n_j)        */
    double energy_after;     /* E_tot^{n+1}, the same sum over the new state       */
    double boundary_flux_dt; /* dt sum_p omega_p mu_p (O*_{N,p} - O*_{0,p}): the
                                net outflow through the two ends, with the
                                prediction's O* (the correction's moment
                                equation (4.13) uses D from O*)                   */
    double energy_defect;    /* energy_after - energy_before + boundary_flux_dt:
                                the defect of (3.13), sum_j dx (rho^{n+1}_j -
                                rho~_j) / c up to rounding; it vanishes with eps */
} grte_step_info;

/* Error flags of the steps since the last clear (grte_get_error_flags): the
 * per-step counters of grte_step_info are reset by every step, these are not. */
enum {
    GRTE_ERRF_SYNC = 1,          /* a grid barrier of the prediction timed out  */
    GRTE_ERRF_PRED_NOCONV = 2,   /* a prediction solve stopped at its cap       */
    GRTE_ERRF_NEWTON = 4,        /* a Newton solve stopped at its cap           */
    GRTE_ERRF_NEGATIVE_ROOT = 8  /* a cell's temperature equation had no root >= 0 */
};

/* Stages readable after a step (grte_get_stage), for checking and diagnostics. */
enum {
    GRTE_STAGE_ESTAR = 0, /* E* of the prediction, N*P, cell-major               */
    GRTE_STAGE_OSTAR = 1, /* O* of the prediction, (N+1)*P, cell-major           */
    GRTE_STAGE_USTAR = 2, /* U* from (4.5c), N                                   */
    GRTE_STAGE_D = 3,     /* flux divergence D of (4.13), N                      */
    GRTE_STAGE_RHO = 4    /* rho^{n+1} = sum_p omega_p E^{n+1}_p, N              */
};

/* Gauss-Legendre parity pairs (host, no device work): the nv/2 positive
 * nodes of the nv-point rule on [-1, 1] in increasing order, and the weight of
 * +mu_p, so that sum_p omega_p = 1 and rho = sum_p omega_p E_p.  nv even,
 * 2 <= nv <= 128; mu and omega must hold nv/2 doubles.  (The paper leaves the
 * velocity grid open; see the remark after (4.5).) */
grte_status grte_gauss_legendre(int nv, double *mu, double *omega);

/* Create a context: copies the problem and the velocity grid (host arrays
 * mu[P], omega[P] with mu_p > 0; the exact binary64 weights are used, their
 * sum need not be exactly one) and allocates device memory.  The state is
 * zero and the opacity one until set.  *out receives the context. */
grte_status grte_create(const grte_problem *pb, const double *mu,
                        const double *omega, grte_ctx **out);

/* Free the context and its device memory (NULL is accepted). */
grte_status grte_destroy(grte_ctx *ctx);

/* Order all further work of the context on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  The stream must outlive its use. */
grte_status grte_set_stream(grte_ctx *ctx, void *hip_stream);

/* Opacity coefficient per cell: sigma0[N] >= 0 ((1.1), or the T-independent
 * factor of sigma/T^3 in (1.4)). */
grte_status grte_set_opacity(grte_ctx *ctx, const double *sigma0, int on_device);

/* Inflow data (4.1): b_left[p] = b_L(mu_p) at x = 0, b_right[p] = b_R(-mu_p)
 * at x = L; host arrays of P doubles. */
grte_status grte_set_inflow(grte_ctx *ctx, const double *b_left, const double *b_right);

/* State (E^n, O^n, T^n): E[N*P], O[(N+1)*P] cell-major, T[N] >= 0. */
grte_status grte_set_state(grte_ctx *ctx, const double *E, const double *O,
                           const double *T, int on_device);

/* Copy the current state out (same layouts as grte_set_state).  Any of the
 * three pointers may be NULL to skip it. */
grte_status grte_get_state(grte_ctx *ctx, double *E, double *O, double *T, int on_device);

/* Cell-centre intensities of the current state: I[j*2P + p] = I(+mu_p) and
 * I[j*2P + P + p] = I(-mu_p), i.e. E_{j,p} + eps (O_{j,p} + O_{j+1,p})/2 and
 * E_{j,p} - eps (O_{j,p} + O_{j+1,p})/2: the parities (4.2) with O interpolated to
 * the cell centre as in the inflow relations (4.6); eps > 0 the scaling of the
 * state.  I holds 2 N P doubles
 * (host or device).  With binary32 storage, of the stored state. */
grte_status grte_get_intensity(grte_ctx *ctx, double eps, double *I, int on_device);

/* One AP step of Algorithm 2 with time step dt > 0 and eps > 0.  The state is
 * replaced by (E^{n+1}, O^{n+1}, T^{n+1}).  With info == NULL the call only
 * enqueues work; otherwise it synchronises and fills *info.  Returns
 * GRTE_E_NOCONV (state still advanced) if info != NULL and a solve hit its
 * cap.  The prediction's iteration starts from rho^n = sum_p omega_p E^n_p,
 * or, when the current state is the one the previous grte_step /
 * grte_step_group of ctx produced, from that step's converged rho* (fewer
 * iterations; the converged result is the same to the solver tolerance).
 * grte_set_state, grte_set_storage and grte_reference_step return to rho^n. */
grte_status grte_step(grte_ctx *ctx, double dt, double eps, grte_step_info *info);

/* One AP step of n independent contexts with one launch of each kernel
 * (1 <= n <= 4; the contexts must be distinct, on one device and of the same
 * tile shape, i.e. the same rows per thread: N in the same one of the ranges
 * (0,512], (512,1024], (1024,2048], (2048,4096]).  Context g advances with
 * dt[g], eps[g]; the results are those of n separate grte_step calls, bit for
 * bit.  All work is ordered on the first context's stream (the caller orders
 * the others' streams with it).  info (n entries) as for grte_step; the
 * status is the worst over the contexts.  GRTE_E_UNSUPPORTED if the pairs of
 * all contexts exceed the device's co-resident work-groups. */
grte_status grte_step_group(grte_ctx *const *ctxs, int n, const double *dt, const double *eps,
                            grte_step_info *info);

/* The iterative implicit reference solver of the paper's nonlinear-opacity
 * examples, (6.6): backward Euler in I and U with the opacity sigma0/T^3
 * frozen at the previous iterate T^(k) = (U^(k))^(1/4), iterated from
 * T^(0) = T^n until max|T^(k+1) - T^(k)| <= tol max T^(k+1) (at most maxit
 * times).  On the parity grid one iteration is the prediction system (5.2)
 * with K from T^(k); at the fixed point E^{n+1} = E*, O^{n+1} = O*,
 * U^{n+1} = U*.  Replaces the state like grte_step; synchronises.
 * GRTE_E_NOCONV if the iteration (or a prediction solve) hit its cap;
 * GRTE_E_UNSUPPORTED with binary32 storage. */
typedef struct grte_reference_info {
    int picard_iters, converged, pred_max_iters, pred_failed, sync_error;
} grte_reference_info;
grte_status grte_reference_step(grte_ctx *ctx, double dt, double eps, double tol, int maxit,
                                grte_reference_info *info);

/* How the prediction kernel is launched.  Its work-groups (one per parity
 * pair, over all contexts of a grouped step) wait for each other at grid
 * barriers inside the kernel, so all of them must be resident at once.
 * cooperative = 1 (default): a cooperative launch, for which the runtime
 * guarantees that.  cooperative = 0: an ordinary launch of the same grid,
 * ~18 us faster per step on an MI355X; it relies on the grid fitting the
 * device at once (checked at creation against the kernel's occupancy, as for
 * the cooperative launch) and on no other work -- another stream, another
 * process -- holding the device's compute units while the step runs.  For
 * callers that own the device.  If the assumption fails, the barriers' bounded
 * wait expires and the step reports sync_error (GRTE_E_HIP when info is
 * requested) with invalid results; it never hangs.  The setting of the first
 * context applies to a grouped step; the implicit reference step uses its
 * context's.  GRTE_E_INVAL for a null ctx or a value other than 0 or 1. */
grte_status grte_set_launch(grte_ctx *ctx, int cooperative);

/* Correction stage of the step.
 * GRTE_CORRECTION_CONSERVATIVE (default): Algorithm 2's correction, (4.13)
 *   by a scalar Newton per cell, then (4.11)+(4.12), projection (4.14).
 * GRTE_CORRECTION_ALT: the alternative of the remark closing Section 3,
 *   (3.14): the time derivative of the intensity taken from the prediction's
 *   update and the emission at U*, which needs no nonlinear solve -- per
 *   direction (4.11a,b) with U^{n+1} -> U* and the known time-derivative
 *   terms (K = (T^n)^m), then T^{n+1} = T^n + dt sigma0 rho_J / (eps K Cv)
 *   explicitly, then (4.14).  The remark reports it not energy conservative
 *   (the step's energy_defect does not vanish with eps; boundary_flux_dt is
 *   then formed with the correction's O_J) and failing for T-dependent
 *   opacity; it is kept as the ablation the remark describes.  Needs
 *   sigma0 > 0 in every cell (it divides by the node opacity) and binary64
 *   storage (GRTE_E_UNSUPPORTED with binary32, either way round).  A grouped
 *   step needs the same kind in every context (GRTE_E_INVAL otherwise). */
enum { GRTE_CORRECTION_CONSERVATIVE = 0, GRTE_CORRECTION_ALT = 1 };
grte_status grte_set_correction(grte_ctx *ctx, int kind);

/* The GRTE_ERRF_* flags OR-ed over every step since the context was created
 * or the flags were last cleared (clear != 0 clears them after reading).
 * Lets a caller that enqueues many steps without `info` (no host
 * synchronisation per step) check afterwards that none of them timed out at a
 * grid barrier or stopped at an iteration cap.  Synchronises the stream. */
grte_status grte_get_error_flags(grte_ctx *ctx, int *flags, int clear);

/* Storage of the intensity state: 0 = binary64 (default); 1 = binary32, with
 * E kept per cell and pair as its binary32 deviation from a c T^4 (T stays
 * binary64) and O in binary32.  The prediction, Newton and correction
 * arithmetic, the angular sums (binary64 accumulation of the widened
 * values) and T stay binary64; only the stored E and O are rounded, once per
 * step.  The current state is converted; grte_set_state / grte_get_state keep
 * exchanging binary64 arrays (get_state returns the values the binary32
 * storage represents). */
grte_status grte_set_storage(grte_ctx *ctx, int fp32);

/* Convergence history of the last prediction solve of ctx (of a grte_step,
 * grte_step_group or the last Picard sweep of grte_reference_step): entry k is
 * max|z| / max|rho| of update k + 1, the quantity the stopping test compares
 * with pred_tol.  The first GRTE_HIST_CAP updates are kept.  Copies
 * min(cap, updates kept) values to the host array out, sets *n to that count
 * and synchronises the context's stream.  GRTE_E_INVAL for a null ctx or n,
 * a negative cap, or a null out with cap > 0. */
enum { GRTE_HIST_CAP = 1024 };
grte_status grte_get_pred_history(grte_ctx *ctx, double *out, int cap, int *n);

/* Copy a stage of the last step (GRTE_STAGE_*) into out (sizes above). */
grte_status grte_get_stage(grte_ctx *ctx, int stage, double *out, int on_device);

/* Solver controls: relative tolerance of the prediction update (default
 * 1e-15), its iteration cap (default 200) and the Newton cap (default 100).
 * The prediction stops when max|z| <= pred_tol max|rho| for its update z, or,
 * as a safeguard, when the update norm has reached the rounding level of the
 * residual evaluation, where it only fluctuates: max|z| <= 16 pred_tol
 * max|rho| and max|z| / max|rho| has not decreased over the last two updates,
 * or max|z| <= 64 pred_tol max|rho| and max|z| / max|rho| is above 0.9 of its
 * value three updates earlier (that level is about 1e-16 relative on
 * optically thick slabs, e.g. N = 4096, 64 ordinates, eps = 1e-4, and up to
 * ~2.3e-14 on some binary32-stored states of the batched ensemble right after
 * the cold start).  Both count as converged (info pred_converged); the second
 * also sets pred_floor_stop (the batched path applies the same test). */
grte_status grte_set_solver(grte_ctx *ctx, double pred_tol, int pred_maxit, int newton_maxit);

/* Acceleration of the prediction iteration (default GRTE_ACCEL_CHEBYSHEV).
 * Both modes iterate the same DSA-preconditioned update z = res + D^-1 (G res)
 * and stop on the same test max|z| <= pred_tol max|rho|; they differ only in
 * how z is applied:
 *   GRTE_ACCEL_RICHARDSON  rho += z;
 *   GRTE_ACCEL_CHEBYSHEV   plain updates until the contraction ratio r of
 *     the update norms has settled (two consecutive ratios within 15%, r <= 0.5,
 *     update norm above 100 pred_tol max|rho|), then the Chebyshev
 *     semi-iteration for an iteration-matrix spectrum in [0, 1.2 r]; plain
 *     updates for the rest of the solve if, 4 or more steps in, the update norm
 *     is above what plain updates at ratio r would have reached, or above the
 *     norm at which the recurrence began.  No inner products are formed.
 * The converged rho agrees between the modes to the tolerance; iteration
 * counts differ.  GRTE_E_INVAL for another mode. */
enum { GRTE_ACCEL_RICHARDSON = 0, GRTE_ACCEL_CHEBYSHEV = 1 };
grte_status grte_set_acceleration(grte_ctx *ctx, int mode);

/* Stage timing with HIP events recorded on the context's stream around each
 * timed stage of a step (grte_step, or grte_step_group through its first
 * context).  on = 0: off (default); on = k >= 1: every k-th step from now is
 * timed (each event record costs the stream a few microseconds, so sampling
 * keeps the timed run close to an untimed one).  Setting resets the log;
 * GRTE_E_INVAL for on < 0. */
enum {
    GRTE_TIMING_STEP = 0,     /* the whole step, first to last kernel          */
    GRTE_TIMING_PREDICT = 1,  /* the prediction solve kernel (4.5)/(5.2)       */
    GRTE_TIMING_NSTAGES = 2
};
grte_status grte_set_profiling(grte_ctx *ctx, int on);

/* Synchronise the stream and return, per GRTE_TIMING_* stage, the summed
 * elapsed milliseconds and the number of timed launches since profiling was
 * enabled or last read (arrays of GRTE_TIMING_NSTAGES entries); clears the log. */
grte_status grte_read_timing(grte_ctx *ctx, double *total_ms, int *count);

/* ------------------------------------------------------------------------
 * Learned initial guess of the temperature solve (4.13)/(5.5).
 *
 * A multilayer perceptron 5 -> 64 -> 64 -> 1 with exact gelu activations maps
 * f = log10(rho*, T^n, sigma0 (T^n)^-m, eps, dt), standardised with
 * (mu_f, sd_f), to y; the starting value is T0 = T^n exp(mu_t + sd_t y).
 * Inference uses the weights rounded to bfloat16 (nearest even) with binary32
 * accumulation.  Every guess is judged by the normalised residual
 * |alpha T0^4 + T0 - s| / max(|s|, tiny) of (4.13) (alpha T^4 + T - s = 0):
 * at or below the acceptance bound it is the result; otherwise Newton starts
 * from T0 if its residual is below that of T^n.  If T0 is not a positive
 * finite number, is the worse start, or Newton from it hits its cap, plain
 * Newton from T^n decides (grte_step_info counts each case).
 *
 * Parameters: 4609 binary32 values, W1 (64x5 row-major), b1 (64), W2 (64x64,
 * row = output unit), b2 (64), W3 (64), b3 (1).  Normalisation: 12 values
 * mu_f[5], sd_f[5], mu_t, sd_t.  Training rows: 6 binary32 values
 * (f_0..f_4, log(T^{n+1}/T^n)), row-major, device memory.  Training is Adam
 * (beta 0.9/0.999, eps 1e-8) on the mean squared error of the standardised
 * target, binary32 master parameters, minibatches taken in row order
 * (wrapping; shuffle the rows beforehand).
 * ------------------------------------------------------------------------ */
typedef struct grte_mlp grte_mlp;
grte_status grte_mlp_create(grte_mlp **out);        /* zero parameters, unit normalisation */
grte_status grte_mlp_destroy(grte_mlp *m);
grte_status grte_mlp_set_stream(grte_mlp *m, void *hip_stream);
/* Host parameters in (4609); resets the Adam moments and step count. */
grte_status grte_mlp_set_params(grte_mlp *m, const float *theta);
/* Host copies out: binary32 master values and/or their bfloat16 bit patterns
 * (either pointer may be NULL). */
grte_status grte_mlp_get_params(grte_mlp *m, float *theta, unsigned short *theta_bf16);
grte_status grte_mlp_set_norm(grte_mlp *m, const float *norm);   /* 12 host values, sd > 0 */
grte_status grte_mlp_get_norm(grte_mlp *m, float *norm);
/* Normalisation from n >= 2 training rows (column means and standard deviations). */
grte_status grte_mlp_fit_norm(grte_mlp *m, const float *dev_rows, long long n);
/* Loss and gradient (host, 4609) of the mean squared error over n rows. */
grte_status grte_mlp_grad(grte_mlp *m, const float *dev_rows, long long n, float *grad, float *loss);
/* `steps` Adam steps with minibatches of `batch` rows and learning rate lr;
 * loss_hist (host, may be NULL) receives the minibatch loss of each step. */
grte_status grte_mlp_train(grte_mlp *m, const float *dev_rows, long long n, int steps, int batch,
                           float lr, float *loss_hist);
/* The same training as grte_mlp_train, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving or training loops that
 * forbid hipMalloc): it calls no hipMalloc, hipFree or other allocating
 * routine.  Its per-block partial gradients and losses and its loss history
 * live in one fixed workspace of 4.98 MB in the library's code object, which
 * each device holds until the process ends: at most 16384 rows per minibatch
 * (min(batch, n)) and, when loss_hist is non-NULL, at most 65536 steps;
 * larger requests return GRTE_E_UNSUPPORTED (with a message on stderr) and do
 * nothing.  Every call on a device shares that device's workspace: calls that
 * overlap on one device (two streams, two threads) race and must not be made.
 * Results are bit-identical to grte_mlp_train's for the same model state,
 * rows and arguments (the same kernels in the same order).  Synchronises the
 * model's stream. */
grte_status grte_mlp_train_noalloc(grte_mlp *m, const float *dev_rows, long long n, int steps, int batch,
                                   float lr, float *loss_hist);
/* Network outputs y (device, n) for the feature columns of n rows. */
grte_status grte_mlp_predict(grte_mlp *m, const float *dev_rows, long long n, float *dev_y);
/* Use `model` (NULL: plain Newton from T^n) for the temperature solve of
 * later steps of ctx, with acceptance bound accept_tol (e.g. 1e-10).  The
 * model is borrowed: it must outlive its use and not be trained meanwhile. */
grte_status grte_set_guess(grte_ctx *ctx, const grte_mlp *model, double accept_tol);
/* Training rows of the last step (one per cell, N rows) into dev_rows
 * (capacity cap_rows >= N); cells with sigma0 = 0 give a zero row.  Requires a
 * step since the last grte_set_state.  Enqueued on the context's stream. */
grte_status grte_log_pairs(grte_ctx *ctx, float *dev_rows, long long cap_rows, long long *n_rows);

/* ------------------------------------------------------------------------
 * The discrete nonlinear diffusion limit on the GPU: the three-stage scheme
 * (2.7) (sigma independent of T) and its sigma0/T^3 form (2.9), the two-stage
 * scheme (2.8) and the limit of the alternative correction (3.14).  State T per cell (N <= 4096) on the cell-centred
 * grid of the AP step; face coefficients a c K/(3 sigma) with the harmonic
 * mean of sigma0 and the mean of K = T^m of the two cells.  Boundaries:
 * 0 = zero flux, 1 = ghost temperatures one cell outside each end (the
 * boundary cell's coefficient on the boundary face).
 * ------------------------------------------------------------------------ */
typedef struct grte_diff grte_diff;
typedef struct grte_diff_problem {
    int nx;                   /* cells, 2 <= N <= 4096                            */
    double length, a, c, cv;
    int opacity_law;          /* 0: sigma = sigma0; 3: sigma = sigma0 / T^3       */
    int boundary;             /* 0: zero flux; 1: ghost temperatures              */
    double ghost_left, ghost_right;
} grte_diff_problem;
/* GRTE_DIFF_SEMI_COR: the diffusion limit printed for the alternative correction
 * (3.14) (remark closing Section 3): the prediction of (2.7)/(2.9), then the
 * linear update a (U* - U^n)/dt + Cv (T^{n+1} - T^n)/dt = div(F^n grad U*) --
 * no Newton solve, not energy-conservative, only conditionally stable. */
enum { GRTE_DIFF_THREE_STAGE = 0, GRTE_DIFF_TWO_STAGE = 1, GRTE_DIFF_SEMI_COR = 2 };
grte_status grte_diff_create(const grte_diff_problem *pb, grte_diff **out);
grte_status grte_diff_destroy(grte_diff *d);
grte_status grte_diff_set_stream(grte_diff *d, void *hip_stream);
grte_status grte_diff_set_opacity(grte_diff *d, const double *sigma0, int on_device);  /* > 0 */
grte_status grte_diff_set_state(grte_diff *d, const double *T, int on_device);         /* T >= 0 */
/* T^{n} after the last step and U* of its prediction (either may be NULL). */
grte_status grte_diff_get_state(grte_diff *d, double *T, double *Ustar, int on_device);
/* One step.  scheme: GRTE_DIFF_*; corr_K (sigma0/T^3 only): 0 = the correction
 * flux with K^n (the limit of the AP step), 1 = with (U*)^{3/4} as printed in
 * (2.9); a_time < 0: a, otherwise a_time replaces a in the time-derivative
 * terms (a_time = 0 gives a porous-medium equation).  newton_its (may be NULL;
 * then the call only enqueues): largest Newton count; GRTE_E_NOCONV at the cap. */
grte_status grte_diff_step(grte_diff *d, double dt, int scheme, int corr_K, double a_time, int *newton_its);

/* Static text for a status code. */
const char *grte_status_string(grte_status s);

/* ------------------------------------------------------------------------
 * Batched slabs: many independent 1-D problems of the kind above, each with
 * its own N, P, opacity law, eps and dt, advanced together by one persistent
 * kernel per step (one tile of 256 or 64 threads per instance, instances
 * taken from a device work queue in longest-first order).  Each instance
 * computes exactly the step of grte_step (Algorithm 2).
 *
 * Packed layouts: instances are concatenated in the order given at creation.
 * For instance i with N_i cells and P_i pairs, its block starts at
 *   cells:  sum_{k<i} N_k            (T, sigma0)
 *   E:      sum_{k<i} N_k P_k        (E[j*P_i + p] inside the block)
 *   O:      sum_{k<i} (N_k + 1) P_k  (O[i*P_i + p] inside the block)
 *   pairs:  sum_{k<i} P_k            (mu, omega, inflow data)
 * grte_batch_sizes returns the four totals.  Limits: 2 <= N_i <= 2048,
 * 1 <= P_i <= 64.  The other conventions are those of the single context.
 * ------------------------------------------------------------------------ */
typedef struct grte_batch grte_batch;

typedef struct grte_instance {
    int nx;            /* cells N_i                                             */
    int npairs;        /* parity pairs P_i                                      */
    int opacity_law;   /* 0 or 3, as grte_problem.opacity_law                   */
    double length, a, c, cv;
    double dt, eps;    /* time step and eps of this instance (fixed)            */
} grte_instance;

typedef struct grte_batch_info {   /* per instance, as grte_step_info         */
    int pred_iters, pred_converged, newton_max_iters, newton_failed;
    int kstar_clamped, negative_root;
    int pred_floor_stop;
    /* energy balance of the instance's step, (3.12)-(3.13), as in
     * grte_step_info (binary64, fixed summation order for a given tile) */
    double energy_before, energy_after, boundary_flux_dt, energy_defect;
} grte_batch_info;

typedef struct grte_batch_tuning {
    int wave_max_n;    /* instances with N <= wave_max_n (<= 256) run on one
                          wavefront, the others on a 256-thread work-group    */
    int grid;          /* work-groups of the persistent launch                 */
    double step_ms;    /* filled by grte_batch_tune: time of one step          */
} grte_batch_tuning;

/* Create a batch of n instances; mu/omega are packed per-instance velocity
 * grids (P_i entries each, mu > 0, omega > 0).  State zero, opacity one,
 * inflow zero until set.  Returns GRTE_E_UNSUPPORTED beyond the limits. */
grte_status grte_batch_create(int n, const grte_instance *inst, const double *mu,
                              const double *omega, grte_batch **out);
grte_status grte_batch_destroy(grte_batch *b);
/* Totals of the packed layouts (any pointer may be NULL). */
grte_status grte_batch_sizes(const grte_batch *b, long long *cells, long long *e_len,
                             long long *o_len, long long *pairs);
grte_status grte_batch_set_stream(grte_batch *b, void *hip_stream);
grte_status grte_batch_set_solver(grte_batch *b, double pred_tol, int pred_maxit, int newton_maxit);
/* Binary32 storage of every instance's intensity state, as grte_set_storage
 * for one slab: with fp32 = 1 the stored E is fl32(E - a c T^4) (T of the same
 * state) and O is fl32(O); every step computes in binary64 from the stored
 * values and rounds its result once.  The current state is converted;
 * grte_batch_set_state / grte_batch_get_state keep exchanging binary64 packed
 * arrays (get_state returns the values the binary32 storage represents).  A
 * captured step graph is rebuilt.  GRTE_E_INVAL for fp32 other than 0 or 1,
 * GRTE_E_NOMEM if the binary32 buffers cannot be allocated. */
grte_status grte_batch_set_storage(grte_batch *b, int fp32);
/* Acceleration of the prediction iteration of every instance (GRTE_ACCEL_*,
 * as grte_set_acceleration; default GRTE_ACCEL_CHEBYSHEV).  Takes effect at
 * the next step (a captured step graph is rebuilt). */
grte_status grte_batch_set_acceleration(grte_batch *b, int mode);
/* Packed sigma0[cells]; packed inflow b_left[pairs], b_right[pairs] (host). */
grte_status grte_batch_set_opacity(grte_batch *b, const double *sigma0, int on_device);
grte_status grte_batch_set_inflow(grte_batch *b, const double *b_left, const double *b_right);
/* Packed state E[e_len], O[o_len], T[cells] in and out. */
grte_status grte_batch_set_state(grte_batch *b, const double *E, const double *O,
                                 const double *T, int on_device);
grte_status grte_batch_get_state(grte_batch *b, double *E, double *O, double *T, int on_device);
/* One step of every instance.  info == NULL: enqueue only; otherwise
 * synchronise and fill info[n]; GRTE_E_NOCONV if any instance hit a cap.
 * As for grte_step, each prediction starts from the instance's rho* of the
 * previous step when the current state is the one that step produced
 * (grte_batch_set_state and grte_batch_set_storage return to rho^n). */
grte_status grte_batch_step(grte_batch *b, grte_batch_info *info);
/* GRTE_ERRF_* flags OR-ed over every step (of any instance) since creation or
 * the last clear, as grte_get_error_flags: PRED_NOCONV, NEWTON and
 * NEGATIVE_ROOT (the batched step has no grid barrier).  For callers that
 * enqueue steps or graph replays without `info`.  Synchronises the stream. */
grte_status grte_batch_get_error_flags(grte_batch *b, int *flags, int clear);
/* Autotuner: times `trials` steps for each candidate (wavefront threshold
 * 0/128/256 x grid of 1, 2, ... work-groups per compute unit) from the
 * current state without changing it (each candidate step also starts its
 * prediction from the same iterate as the next real step will), orders the
 * instances by the measured work (iterations x N x P, largest first) and
 * keeps the fastest choice.  Tune on a state like the ones to be stepped
 * through: the cold start needs a fraction of a developed state's iterations. */
grte_status grte_batch_tune(grte_batch *b, int trials, grte_batch_tuning *best);
grte_status grte_batch_set_tuning(grte_batch *b, const grte_batch_tuning *t);
grte_status grte_batch_get_tuning(const grte_batch *b, grte_batch_tuning *t);
/* on != 0: every step replays a captured HIP graph (one per state-buffer
 * parity, captured at first use and after any change of tuning or solver). */
grte_status grte_batch_use_graph(grte_batch *b, int on);
/* Event timing on the batch stream.  While profiling is on, every step runs
 * its kernels as direct launches (not a graph replay) with HIP events around
 * the whole step and around its prediction-solve kernel (the per-slab solves
 * of (4.5), the step's dominant kernel).  grte_batch_read_timing returns the
 * summed step milliseconds and the number of steps since the last read;
 * grte_batch_read_timing2 also the summed prediction-solve milliseconds.  Both
 * synchronise the batch stream and start a new count. */
grte_status grte_batch_set_profiling(grte_batch *b, int on);
grte_status grte_batch_read_timing(grte_batch *b, double *total_ms, int *count);
grte_status grte_batch_read_timing2(grte_batch *b, double *step_ms, double *solve_ms, int *count);

/* ===========================================================================
 * The AP step on a 2-D rectangle [0, lx] x [0, ly] (nx x ny cells).
 *
 * The paper's scheme is one-dimensional; this is its extension on a staggered
 * parity grid: E_p in the cells, the odd parity O_p on the faces (O^x on the
 * x-faces, O^y on the y-faces), the O-equation of (4.3) at every interior face
 * with Omega_p . grad E discretised as the compact difference across the face
 * plus the mean of the two adjacent cells' centred differences along the face
 * (one-sided at a wall), the E-equation in every cell with the discrete
 * divergence, and the inflow relation (4.6) at the centre of every edge cell
 * through the cell's two faces normal to the edge.  Each step is Algorithm 2:
 * prediction (4.5)/(5.2), the scalar equation (4.13) per cell, correction
 * (4.11)-(4.12), projection (4.14).  Both linear systems are solved by a
 * preconditioned Krylov method to a relative residual (grte2d_set_solver).
 *
 * Layouts (binary64, cell-major, pair index fastest; device or host):
 *   E[(iy*nx + ix)*P + p]        cells, ix along x, iy along y
 *   Ox[(iy*(nx+1) + fx)*P + p]   x-faces fx = 0..nx (face fx between cells fx-1, fx)
 *   Oy[(fy*nx + ix)*P + p]       y-faces fy = 0..ny
 *   T[iy*nx + ix], sigma0[iy*nx + ix]
 * Direction pair p: Omega_p = (mu_p, eta_p) with eta_p > 0 and mu_p != 0 (no
 * direction parallel to an edge), and -Omega_p; omega_p the pair weight,
 * rho = sum_p omega_p E_p.
 * ======================================================================== */
typedef struct grte2d_ctx grte2d_ctx;

typedef struct grte2d_problem {
    int nx, ny;        /* cells along x and y, each >= 2; nx*ny <= 2^28 and      
                          (nx+1)*(ny+1)*npairs < 2^31 (32-bit indexing)        */
    int npairs;        /* P: a power of two, 1 <= P <= 64                        */
    double lx, ly;     /* rectangle sides > 0                                    */
    double a, c, cv;   /* radiation constant, speed of light, heat capacity > 0  */
    int opacity_law;   /* m: 0 -> sigma = sigma0; 3 -> sigma = sigma0 / T^3      */
} grte2d_problem;

typedef struct grte2d_step_info {
    int pred_iters;          /* Krylov iterations of the prediction               */
    int pred_converged;      /* 1 if its true relative residual met the tolerance */
    double pred_residual;    /* that residual, ||b - A x||_2 / ||b||_2             */
    int corr_iters;          /* the same for the correction                        */
    int corr_converged;
    double corr_residual;
    int newton_max_iters;    /* largest Newton iteration count over the cells     */
    int newton_failed;       /* cells whose Newton solve hit the cap               */
    int kstar_clamped;       /* sigma/T^3: cells with U* < 0 (K* taken as 0)       */
    int negative_root;       /* cells whose (4.13) has no root >= 0                */
    int newton_total_iters;  /* Newton iterations summed over the cells            */
    int guess_accepted;      /* learned guess (grte2d_set_guess): cells whose guess
                                met the residual bound (no Newton step)            */
    int guess_rejected;      /* cells whose guess was unusable, no better than T^n
                                by residual, or whose Newton from it hit the cap  */
    int guess_started;       /* cells whose Newton started from the guess          */
    int pred_floor_stop;     /* 1 if a solve was accepted at the rounding level of */
    int corr_floor_stop;     /* its residual: restarting no longer reduced it and
                                it was within 64 x max(tol, that level), the level
                                being 2^-53 || |A| |x| + |b| ||_2 / ||b||_2 (the
                                normwise backward-error floor of a binary64
                                iterate; counted in *_converged)                   */
    /* Energy balance of the step, (3.12)-(3.13) on the rectangle: binary64
     * sums in a fixed order, formed on the device every step (values of the
     * binary64 state, before a binary32 storage rounds it). */
    double energy_before;    /* E_tot^n = sum_cells dx dy (rho^n / c + Cv T^n)    */
    double energy_after;     /* E_tot^{n+1}                                       */
    double boundary_flux_dt; /* dt x the net outflow through the four edges: dy
                                sum_rows sum_p omega_p mu_p (O*x_right - O*x_left)
                                + dx sum_cols sum_p omega_p eta_p (O*y_top -
                                O*y_bottom), the prediction's edge face values    */
    double energy_defect;    /* energy_after - energy_before + boundary_flux_dt:
                                the defect of (3.13)                              */
    int pred_narrow;         /* 1 if the prediction's Krylov vectors were stored in
                                binary32 (grte2d_set_krylov_storage)              */
    int corr_narrow;         /* the same for the correction                        */
} grte2d_step_info;

enum {
    GRTE2D_STAGE_ESTAR = 0,  /* E* of the prediction, nx*ny*P                     */
    GRTE2D_STAGE_USTAR = 1,  /* U* from (4.5c), nx*ny                              */
    GRTE2D_STAGE_D = 2,      /* flux divergence D of (4.13), nx*ny                 */
    GRTE2D_STAGE_RHON = 3    /* rho^n = sum_p omega_p E^n_p, nx*ny                 */
};

/* nv equally spaced directions theta_k = 2 pi (k + 1/2)/nv on the unit circle
 * (host, no device work): the nv/2 pairs k < nv/2 with mu = cos, eta = sin,
 * omega = 2/nv.  nv a multiple of 4, 4 <= nv <= 128; arrays of nv/2 doubles. */
grte_status grte2d_circle_directions(int nv, double *mu, double *eta, double *omega);

/* Create a context: copies the problem and the pairs (host arrays of P doubles)
 * and allocates device memory (about 16 binary64 arrays of nx*ny*P).  State
 * zero, opacity one, inflow zero until set.  GRTE_E_UNSUPPORTED for sizes or P
 * outside the limits above, GRTE_E_INVAL for bad values, GRTE_E_NOMEM. */
grte_status grte2d_create(const grte2d_problem *pb, const double *mu, const double *eta,
                          const double *omega, grte2d_ctx **out);

/* Free the context (NULL accepted). */
grte_status grte2d_destroy(grte2d_ctx *ctx);

/* Order the context's work on `hip_stream` (NULL = the null stream). */
grte_status grte2d_set_stream(grte2d_ctx *ctx, void *hip_stream);

/* Krylov tolerance on the relative 2-norm residual (default 1e-14) and the
 * iteration cap per solve (default 2000).  The residual is recomputed from the
 * equations (in a form whose rounding stays near the residual's own size)
 * after each pass of iterations, and the solve restarted from it, up to six
 * times; an iterate whose residual no longer drops by half from one pass to
 * the next is accepted when within 64 x max(tol, the residual's rounding
 * level) -- stiff problems (a c beta of (4.5c) above ~1e7) cannot reach
 * 1e-14. */
grte_status grte2d_set_solver(grte2d_ctx *ctx, double tol, int maxit);

/* Launch shape of the Krylov kernels: each thread takes `items_per_thread`
 * (cell, pair) items (1..64, default 4; at most 16384 blocks of 256 threads),
 * and the per-block partial sums of the inner products are reduced in two
 * levels when there are more than `first_level` of them (1..16384, default
 * 16384: blocks of that many partials, then one block), else by one block of
 * 1024 threads.  The
 * results differ only in the order of the binary64 sums.  A small shape makes
 * a small grid run the many-block, two-level path of a large one (tests).
 * GRTE_E_INVAL outside those ranges. */
grte_status grte2d_set_launch_shape(grte2d_ctx *ctx, int items_per_thread, int first_level);

/* Storage of the Krylov vectors (r, p, B^-1 p, A B^-1 p, s, B^-1 s, A B^-1 s and
 * the block inverse's 1/d_p; the arithmetic is binary64 either way).
 * narrow = 1 (the default): binary32 where the solve allows it, else binary64;
 * narrow = 0: always binary64.  The iterate x and the true residual b - A x,
 * recomputed from the equations at the start of every pass, are binary64.
 * With binary32 vectors a pass ends once the recursion has reduced its
 * residual to 1e-5 of the pass's starting true residual or to a tenth of the
 * tolerance, so that a solve takes several passes.  The prediction keeps
 * binary64 vectors when some cell's block inverse (diagonal plus the rank-one
 * angular coupling g of (4.5c)) has a Sherman-Morrison denominator
 * 1 - g sum_p omega_p / d_p below 1e-8: it falls like 1 / (a c beta) in stiff
 * cells, where binary32 directions lose the near-isotropic mode the inverse
 * amplifies (just above that level they take more iterations than binary64
 * ones, each cheaper).  The correction's blocks are diagonal.  The info struct
 * reports the storage each solve used.  GRTE_E_INVAL for a NULL context or
 * narrow not 0 or 1. */
grte_status grte2d_set_krylov_storage(grte2d_ctx *ctx, int narrow);

/* The Krylov preconditioner inverts each cell's P x P block (the direction-
 * diagonal part plus the rank-one angular coupling of (4.5c)) and, in the
 * prediction, adds an isotropic correction: an approximate inverse of the
 * operator's angular average over isotropic fields, a 5-point diffusion
 * operator -- the mode that the angular coupling leaves nearly undamped in
 * optically thick cells (the diffusion limit of Section 3).  kind 0: none;
 * kind 1 (default): `steps` Chebyshev steps (default 19) on the Jacobi-scaled
 * operator, in launches over 32 x 32-cell tiles that take up to 9 stencil
 * steps each with a halo of as many cells (one launch up to 10 steps, two up
 * to 19); kind 2: one multigrid
 * V-cycle (2 x 2 cell aggregates, coarse rows with the children's row sums and
 * half their couplings across each side, `steps` weighted-Jacobi sweeps before
 * and after each coarse correction); kind 3: kind 1's map with one launch per
 * Chebyshev step whatever `steps` (the same result to the bit).
 * 1 <= steps <= 64.  The correction's systems have no
 * angular coupling and use the block inverse alone. */
grte_status grte2d_set_isotropic_correction(grte2d_ctx *ctx, int kind, int steps);

/* Storage of the state between steps: fp32 = 1 keeps E (as its deviation from
 * a c T^4) and O^x, O^y in binary32 -- each step reads the stored values widened
 * to binary64 and all arithmetic, the temperature and the Newton solve stay
 * binary64; fp32 = 0 (default) keeps binary64.  Switching on rounds the current
 * state.  get/set_state keep their binary64 layouts (set_state rounds, get_state
 * returns the stored values).  GRTE_E_NOMEM if the binary32 arrays cannot be
 * allocated. */
grte_status grte2d_set_storage(grte2d_ctx *ctx, int fp32);

/* Learned initial guess of the per-cell temperature solve (4.13), as for the
 * 1-D context (grte_set_guess): the model's bfloat16 weights and normalisation
 * are read at every step (the model must outlive its use; NULL = Newton from
 * T^n).  A guess whose normalised residual is at most accept_tol is taken as
 * the root; otherwise Newton starts from it if its residual is below that of
 * T^n, else from T^n. */
grte_status grte2d_set_guess(grte2d_ctx *ctx, const grte_mlp *model, double accept_tol);

/* Training rows of the last step: for every cell six binary32 values, the
 * five standardisable features of (rho*, T^n, sigma0 (T^n)^-m, eps, dt) and the
 * target log(T^{n+1}/T^n), into the device buffer dev_rows (cap_rows >= nx*ny
 * rows).  Enqueued on the context's stream.  GRTE_E_INVAL before a step. */
grte_status grte2d_log_pairs(grte2d_ctx *ctx, float *dev_rows, long long cap_rows, long long *n_rows);

/* Opacity coefficient per cell, sigma0[nx*ny] >= 0. */
grte_status grte2d_set_opacity(grte2d_ctx *ctx, const double *sigma0, int on_device);

/* Inflow b[4*P] (host): b[e*P + p] is the intensity of whichever of +-Omega_p
 * enters through edge e = 0 (x = 0), 1 (x = lx), 2 (y = 0), 3 (y = ly). */
grte_status grte2d_set_inflow(grte2d_ctx *ctx, const double *b);

/* State (E^n, O^x, O^y, T^n) in the layouts above. */
grte_status grte2d_set_state(grte2d_ctx *ctx, const double *E, const double *Ox, const double *Oy,
                             const double *T, int on_device);
grte_status grte2d_get_state(grte2d_ctx *ctx, double *E, double *Ox, double *Oy, double *T,
                             int on_device);

/* One AP step (dt > 0, eps > 0).  Synchronises the stream (the Krylov loop
 * reads its convergence flag); fills *info when non-NULL.  GRTE_E_NOCONV (state
 * still advanced) if a solve missed its tolerance or a Newton solve its cap. */
grte_status grte2d_step(grte2d_ctx *ctx, double dt, double eps, grte2d_step_info *info);

/* Timing of the operator kernel (the matrix-free product inside the Krylov
 * iterations, the step's dominant kernel): with on != 0, HIP events on the
 * context's stream bracket the first product of every batch of iterations of
 * the solves with binary32 Krylov vectors (grte2d_set_krylov_storage);
 * grte2d_read_timing returns the summed milliseconds and the number of timed
 * launches since the last grte2d_set_profiling call. */
grte_status grte2d_set_profiling(grte2d_ctx *ctx, int on);
grte_status grte2d_read_timing(grte2d_ctx *ctx, double *ms, int *count);

/* Cell-centre intensities of the current state: I[c*2P + p] = I(+Omega_p) and
 * I[c*2P + P + p] = I(-Omega_p) for cell c = iy*nx + ix, E_p +- eps O_p with O at
 * the cell centre the mean of the cell's four face values; eps > 0 the scaling
 * of the state.  I holds 2 nx ny P doubles (host or device). */
grte_status grte2d_get_intensity(grte2d_ctx *ctx, double eps, double *I, int on_device);

/* A stage of the last step (GRTE2D_STAGE_*). */
grte_status grte2d_get_stage(grte2d_ctx *ctx, int which, double *out, int on_device);

#ifdef __cplusplus
}
#endif

#endif /* GRTE_H */
