/*
 * sph.h -- C ABI of the MI355X (gfx950) grad-h SPH hot path.
 *
 * The library evaluates, for one set of N particles in 3D, the steps of the
 * SPH main loop described in the GANDALF paper (Hubber, Rosotti & Booth 2017,
 * arXiv:1709.04488, sections 2.1 and 5.1):
 *
 *   neighbour search  -- a Morton-key radix sort and a leaf/box tree over the
 *                        sorted particles (the paper's KD-tree with N_LEAF
 *                        particles per leaf and smoothing-sphere extent boxes,
 *                        section 4.2, rebuilt for the GPU)
 *   density loop      -- rho_i = sum_j m_j W(r_ij, h_i) (eq. EQN:SPHRHO) with
 *                        h_i = eta (m_i/rho_i)^(1/3) (eq. EQN:HRHO) solved by
 *                        Newton-Raphson, Omega_i (eq. EQN:OMEGA), the ideal-gas
 *                        pressure P = (gamma-1) rho u and sound speed
 *   force loop        -- grad-h momentum and energy equations (eqs.
 *                        EQN:GRADHMOMEQN, EQN:GRADHENEQN) with Monaghan
 *                        artificial viscosity (eqs. EQN:MON97ARTVISC,
 *                        EQN:MON97ENERGYDISS) and optional artificial
 *                        conductivity (EQN:MON97ENERGYDISS), the signal speed
 *                        and the CFL time-step (eq. EQN:SPH_DT)
 *   time integration  -- kick-drift-kick leapfrog (eqs. EQN:LFKDK1/EQN:LFKDK2)
 *
 * Kernel (section 2 names two, selected by sph_params.kernel): the M4 cubic
 * spline, support R h with R = 2, W = (1/pi) h^-3 f(r/h),
 *   f(q) = (2-q)_+^3 / 4 - (1-q)_+^3;
 * or the quintic spline (Morris 1996), R = 3, W = (1/(120 pi)) h^-3 f(r/h),
 *   f(q) = (3-q)_+^5 - 6 (2-q)_+^5 + 15 (1-q)_+^5.
 * "R h" below is that support radius.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Particle arrays are structure-of-arrays, one value per particle,
 *           in the caller's index order, and live in DEVICE memory on the
 *           device that was current when the context was created.  The caller
 *           owns them; the library never frees or keeps them past the call
 *           except where stated.  The library owns its context and all scratch
 *           memory (sort buffers, sorted copies, tree, status word), allocated
 *           at most up to the HBM budget given to sph_create.
 * Streams.  Every call enqueues work on the context's HIP stream and returns
 *           without waiting, unless stated otherwise.  Results are valid after
 *           the stream has drained (sph_sync, or any later stream-ordered use).
 *           Exception: a call that needs more capacity than the context holds
 *           (its first call, a larger n, or a smaller leaf_size than before)
 *           first waits for the stream, then frees and reallocates the
 *           context's buffers.  A context sized once by a call at its largest
 *           n and leaf size never waits again; sph_evaluate_noalloc never
 *           allocates at all.
 *           The library issues nothing on the null stream for a context bound
 *           to another stream, so contexts on separate (non-blocking) streams
 *           run concurrently without ordering against each other.
 * Errors.   Argument errors are returned at once (SPH_EINVAL).  Conditions the
 *           device detects (non-finite values, an h solve that did not
 *           converge, a smoothing length too large for the periodic box) are
 *           recorded in a sticky status word and returned by sph_sync.  The
 *           library never aborts and throws nothing across the ABI.
 *           sph_last_error gives a readable description of the last error.
 * Threads.  A context is not thread-safe; distinct contexts are independent.
 * Units.    Any consistent set; the parameters are dimensionless.
 */
#ifndef SPH_MI355X_H
#define SPH_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPH_OK = 0,
    SPH_EINVAL = -1,        /* bad argument (NULL array, n < 0, bad parameter) */
    SPH_ENOMEM = -2,        /* device allocation failed */
    SPH_EDEVICE = -3,       /* a HIP runtime call failed */
    SPH_ENOTCONVERGED = -4, /* some h_i did not reach h_rtol in h_max_iter steps */
    SPH_ESTENCIL = -5,      /* periodic box: some R h_i >= L/2 (minimum image ambiguous) */
    SPH_ENONFINITE = -6,    /* a NaN or Inf input or result */
    SPH_EBUDGET = -7,       /* the working set would exceed the HBM budget */
    SPH_ECAP = -8,          /* an output capacity given by the caller is too small */
    SPH_ESTATE = -9,        /* call out of order (e.g. sph_step before upload) */
    SPH_ELEVEL = -10        /* block time-steps: a particle needs a level deeper than
                               block_lmax */
} sph_status;

enum { SPH_FP64 = 0, SPH_FP32_PAIR = 1 };

/* artificial-conductivity signal speed v'_SIG (section 2.1.1) */
enum { SPH_AC_WADSLEY = 0, SPH_AC_PRICE = 1 };

/* artificial-viscosity switch (section 2.1.1 names both) */
enum { SPH_AV_NONE = 0, SPH_AV_MM97 = 1, SPH_AV_CD10 = 2 };

/* smoothing kernel (section 2): M4 cubic spline (R = 2) or quintic spline (R = 3) */
enum { SPH_KERNEL_M4 = 0, SPH_KERNEL_QUINTIC = 1 };

/*
 * Method parameters.  Defaults (sph_default_params): eta = 1.2 (section
 * 2.1.1), gamma = 5/3, alpha_av = 1, beta_av = 2 alpha_av (section 2.1.1),
 * c_cfl = 0.2 (section 2.1.4), h_rtol = 1e-12, h_max_iter = 50, periodic
 * unit box, FP64, leaf_size 16, no artificial conductivity (alpha_ac = 0,
 * ac_signal = SPH_AC_WADSLEY).
 *
 * Artificial conductivity (second sum of eq. EQN:MON97ENERGYDISS): with
 * alpha_ac > 0 every force pair adds
 *   du_i/dt += (m_j / rhobar_ij) alpha_ac v' (u_i - u_j) rhat_ij . gradW_bar_ij
 * to du/dt (rhobar_ij = (rho_i + rho_j)/2; gradW_bar_ij the mean of the
 * kernel gradients at h_i and h_j, as in the viscosity); accelerations, v_sig
 * and dt do not change.  The kernel rebuilds
 * u_j and P_j from the adiabatic EOS (u = c^2 / (gamma (gamma - 1)),
 * P = rho c^2 / gamma).
 *
 * Artificial-viscosity switches (section 2.1.1 names Morris & Monaghan 1997
 * and Cullen & Dehnen 2010; their published forms): every particle carries
 * its own alpha_i and the viscosity of a pair uses (alpha_i + alpha_j)/2
 * (beta_av stays global).  With av_switch != SPH_AV_NONE the resident state
 * (sph_upload_state / sph_step) evolves alpha, from ps->alpha at upload
 * (NULL: alpha_av for every particle):
 *   SPH_AV_MM97: d alpha/dt = -(alpha - alpha_min) ell c / h
 *                             + max(-div v, 0) (alpha_max - alpha),
 *                integrated by the kick-drift-kick like u (the forces at the
 *                end of a step see the predicted alpha);
 *   SPH_AV_CD10: after the forces at the end of each step (length dt):
 *                A = xi max(-(div v - div v_prev)/dt, 0),
 *                xi = |div v| / (|div v| + |curl v| + 1e-4 c/h),
 *                alpha_loc = max(alpha_max h^2 A / (v_sig^2 + h^2 A), alpha_min),
 *                alpha = alpha_loc if alpha < alpha_loc, else
 *                alpha_loc + (alpha - alpha_loc) exp(-2 ell v_sig dt / h).
 * ell = av_ell, or 0.1 (MM97) / 0.05 (CD10) when av_ell = 0.  div v and
 * curl v are the grad-h SPH estimates
 *   div v_i  = -1/(Omega_i rho_i) sum_j m_j v_ij . grad_i W(r_ij, h_i),
 *   curl v_i = |1/(Omega_i rho_i) sum_j m_j v_ij x grad_i W(r_ij, h_i)|.
 * Stateless sph_forces / sph_evaluate use ps->alpha when it is not NULL and
 * write ps->divv / ps->curlv when those are not NULL, whatever av_switch is.
 *
 * precision = SPH_FP64: every pair term in double precision.
 * precision = SPH_FP32_PAIR: pair separations are formed in single precision
 *   from offsets to each leaf's centre, so their error does not grow with the
 *   distance from the origin; pair arithmetic is single precision; positions,
 *   per-particle accumulators (density sums, h residual, accelerations,
 *   du/dt) and time integration stay double precision.  The single-precision
 *   pair terms leave ~1e-7 relative noise in the h residual, so in this mode
 *   the Newton-Raphson stop tolerance is max(h_rtol, 2e-6).
 */
typedef struct {
    double eta;        /* h = eta (m/rho)^(1/3) */
    double gamma;      /* ratio of specific heats, > 1 */
    double alpha_av;   /* artificial viscosity strength (0 disables it) */
    double beta_av;    /* signal-speed coefficient */
    double c_cfl;      /* CFL multiplier */
    double h_rtol;     /* Newton-Raphson stop: the last step would change h
                          by <= h_rtol h and rho by <= h_rtol rho */
    int32_t h_max_iter;/* Newton-Raphson iteration cap (>= 1) */
    int32_t periodic;  /* 1: periodic box [box_lo, box_hi); 0: isolated */
    double box_lo[3];
    double box_hi[3];
    int32_t precision; /* SPH_FP64 or SPH_FP32_PAIR */
    int32_t leaf_size; /* particles per tree leaf: 8, 16 or 32 */
    double alpha_ac;   /* artificial conductivity strength (>= 0; 0 disables it) */
    int32_t ac_signal; /* SPH_AC_WADSLEY: v' = |v_ij . rhat_ij| (the paper's
                          default); SPH_AC_PRICE: v' = sqrt(|P_i - P_j| / rhobar_ij) */
    int32_t av_switch; /* SPH_AV_NONE (default), SPH_AV_MM97 or SPH_AV_CD10 */
    double alpha_min;  /* switches: floor of alpha (default 0.1) */
    double alpha_max;  /* switches: ceiling of alpha (default 1) */
    double av_ell;     /* switches: decay constant ell (0: 0.1 MM97, 0.05 CD10) */
    int32_t block_lmax; /* 0: one global time-step (sph_step); 1..40: hierarchical block
                           time-steps (sph_substep) with at most this many levels */
    int32_t block_lim;  /* block time-step limiter: force neighbours at most this many
                           levels apart (default 2) */
    int32_t kernel;     /* SPH_KERNEL_M4 (default, R = 2) or SPH_KERNEL_QUINTIC (R = 3) */
    /* Launch shape of the density and force loops (the autotuner's knobs
     * besides leaf_size; neither changes what is computed):
     *   stage_leaves: candidate leaves staged in LDS per step of a sweep,
     *     1..128/leaf_size (0: all 128/leaf_size the LDS tile holds).  The
     *     density results do not depend on it; the force sums may change in
     *     their last bits (the split of a particle's terms over its lanes).
     *   claim_leaves: home leaves a wavefront claims per atomic claim of the
     *     persistent loop, 1..64 (0: 1); results do not depend on it. */
    int32_t stage_leaves;
    int32_t claim_leaves;
    int32_t pad_;       /* zero */
} sph_params;

/*
 * One particle set, device pointers, caller index order.  Which arrays each
 * call reads (R) or writes (W):
 *
 *                     x,y,z  m   h    u    v    rho,omega  pressure,cs  ax..dt  nngb    nforce
 *   sph_build_cells     R          R
 *   sph_density         R      R   RW   (R)       W          W(opt)               W(opt)
 *   sph_forces          R      R   R    R    R    R                       W               W(opt)
 *   sph_evaluate        R      R   RW   R    R    W          W(opt)       W       W(opt)  W(opt)
 *   sph_upload_state    R      R   R    R    R
 *   sph_download_state  W          W    W    W    W(opt)     W(opt)       W(opt)  W(opt)  W(opt)
 *
 * (R): read only when pressure or cs is requested.  v = vx, vy, vz.
 *
 * h on entry to sph_density is the initial guess of each smoothing length
 * (> 0); on return it holds the converged value.  dt is the per-particle
 * CFL step C_CFL h_i / v_sig,i.  (opt) arrays may be NULL.
 */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
    const double *vx, *vy, *vz;
    const double *m;
    const double *u;      /* specific internal energy */
    double *h;            /* smoothing length */
    double *rho, *omega;  /* density, grad-h correction */
    double *pressure, *cs;
    double *ax, *ay, *az; /* dv/dt */
    double *dudt;         /* du/dt */
    double *vsig;         /* max signal speed over force neighbours */
    double *dt;           /* per-particle CFL step */
    int32_t *nngb;        /* density neighbours j != i with r_ij < R h_i */
    int32_t *nforce;      /* force neighbours j != i with r_ij < 2 max(h_i, h_j) */
    double *alpha;        /* optional: per-particle alpha_AV (input; sph_download_state
                             writes the evolved values) */
    double *divv;         /* optional output: velocity divergence */
    double *curlv;        /* optional output: magnitude of the velocity curl */
    int32_t *level;       /* optional output of sph_download_state: time-step level */
} sph_particles;

/* Diagnostics of the last evaluation (stateless or resident). */
typedef struct {
    double time;          /* resident state: sum of the steps taken */
    double dt_last;       /* resident state: step taken by the last sph_step */
    double dt_next;       /* min_i dt_i of the latest forces (next CFL step) */
    double kinetic;       /* sum 1/2 m v^2 (velocities the forces used) */
    double thermal;       /* sum m u */
    double momentum[3];   /* sum m v */
    int64_t steps;        /* resident state: sph_step calls since upload */
    int64_t n_dens_pairs; /* density interactions: sum_i nngb_i at the final h */
    int64_t n_force_pairs;/* force interactions: sum_i nforce_i */
    int64_t dens_pair_evals;  /* density pairs evaluated over all Newton-Raphson iterations */
    int64_t force_pair_evals; /* force pairs evaluated */
    int32_t nr_iter_max;  /* Newton-Raphson iterations of the last density pass (max) */
    int32_t walk_overflows; /* leaves whose neighbour walk overflowed LDS (slow path) */
    int64_t dens_leaf_visits; /* candidate leaves swept by the density loop (all iterations) */
    int64_t dens_walks;   /* tree walks made by the density loop */
    int64_t nr_iter_total;    /* density evaluations summed over particles (mean = / n) */
    /* the next four only while instrumentation bit 1 is set (else 0) */
    int64_t dens_candidate_tests; /* particle-candidate distance tests, density loop */
    int64_t dens_box_tests;   /* particle-leaf box tests, density loop */
    int64_t force_candidate_tests; /* particle-candidate distance tests, force loop */
    int64_t force_box_tests;  /* particle-leaf box tests, force loop */
    int32_t density_walk_overflows; /* of walk_overflows: those of the density loop */
    int32_t force_walk_overflows;   /* of walk_overflows: those of the force loop */
    int64_t dens_list_overflows;    /* particles whose density candidate list outgrew its
                                       capacity in a sweep (swept again at the next Newton step) */
    /* block time-steps (block_lmax > 0) */
    int64_t block_full_steps; /* level-0 steps completed since upload */
    int64_t block_substeps;   /* sub-steps taken since upload */
    int64_t block_active;     /* active particles of the last sub-step */
    int64_t block_updates;    /* active particles summed over the sub-steps */
    double block_time;        /* elapsed time */
    double block_dt_max;      /* length of the current level-0 step */
    int32_t block_synchronised; /* 1 when every particle's step has just ended */
    int32_t pad_;
} sph_state_stats;

typedef struct sph_ctx sph_ctx;

/* Default parameters (see sph_params). */
void sph_default_params(sph_params *p);

/*
 * Create a context bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL = the null stream).  hbm_budget_bytes caps the
 * library's own device allocations (0 = no cap).  *ctx is NULL on error.
 * Initialises its status and scalar words on hip_stream and waits for that.
 */
sph_status sph_create(sph_ctx **ctx, const sph_params *p, void *hip_stream,
                      size_t hbm_budget_bytes);

/* Free everything the context owns.  Waits for its stream.  NULL is a no-op. */
sph_status sph_destroy(sph_ctx *ctx);

/* Rebind the context to another stream: waits for the work already enqueued
 * on the old stream, then subsequent calls enqueue on the new one. */
sph_status sph_set_stream(sph_ctx *ctx, void *hip_stream);

/* Replace the method parameters (same validation as sph_create).  Drops the
 * steps captured by sph_capture_steps (they carry the old parameters), after
 * waiting for the context's stream; capture again to replay. */
sph_status sph_set_params(sph_ctx *ctx, const sph_params *p);

/*
 * Neighbour-search structure for ps (reads x, y, z, h): bounding box, Morton
 * keys, device radix sort, sorted copies of the particle data, leaves of
 * leaf_size consecutive particles with their bounding boxes and largest h, and
 * the tree of boxes above them.  sph_density builds it itself; this entry
 * point exists to time or test the build on its own.
 */
sph_status sph_build_cells(sph_ctx *ctx, const sph_particles *ps);

/*
 * Density loop and h solve (eqs. EQN:SPHRHO, EQN:HRHO, EQN:OMEGA): for each i
 * the h_i with h_i^3 rho_i(h_i) = eta^3 m_i, found by safeguarded
 * Newton-Raphson on h - eta (m_i / rho_i(h))^(1/3) from the guess in ps->h,
 * stopped when the next step would change h_i by at most h_rtol h_i and rho_i
 * by at most h_rtol rho_i (the self term j = i is part of rho_i).  Writes h,
 * rho, omega, and if non-NULL pressure (gamma-1) rho u (reads u then),
 * cs = sqrt(gamma P / rho), nngb.
 * Rebuilds the neighbour structure for the current positions first.
 */
sph_status sph_density(sph_ctx *ctx, sph_particles *ps);

/*
 * Force loop (eqs. EQN:GRADHMOMEQN, EQN:GRADHENEQN, EQN:MON97ARTVISC,
 * EQN:MON97ENERGYDISS, the conductivity term when alpha_ac > 0; signal speed
 * and eq. EQN:SPH_DT).
 * Reads x, y, z, v, m, u, h, rho, omega; writes ax, ay, az, dudt, vsig, dt
 * and, if non-NULL, nforce.  Pairs with r_ij = 0 add nothing to a or du/dt.
 * Reuses the neighbour structure of the last sph_density / sph_build_cells
 * call on the same arrays (same x, y, z pointers and n); otherwise rebuilds.
 */
sph_status sph_forces(sph_ctx *ctx, sph_particles *ps);

/*
 * One full evaluation: the density loop and h solve of sph_density, then the
 * force loop of sph_forces, with the set kept in sorted order on the device
 * in between (one sort and one gather of the inputs, the boxes' largest h
 * refreshed after the h solve instead of a second tree build, one scatter of
 * all outputs).  Reads x, y, z, v, m, u and the guess in h; writes h, rho,
 * omega, ax, ay, az, dudt, vsig, dt and, where non-NULL, pressure, cs, nngb,
 * nforce.  Equals sph_density followed by sph_forces to rounding: neighbour
 * counts and h, rho, omega are identical, the force sums may run in another
 * order.
 */
sph_status sph_evaluate(sph_ctx *ctx, sph_particles *ps);

/*
 * sph_evaluate for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, outputs and errors as sph_evaluate, results bit for bit those of
 * sph_evaluate, but every buffer the call needs beyond the caller's arrays
 * and the context's fixed words (set up by sph_create) lives in one static
 * device array of the library, of fixed size (about 40 MB, held on each
 * device the library runs on until the process ends): the call makes no
 * device allocation or free and never waits for the stream.
 * Limit: n <= sph_noalloc_max_n() (32768); larger n returns SPH_ECAP.
 * The static array is shared by every context on a device and keeps the last
 * call's contents: calls that overlap on one device (other streams, other
 * threads) race and must be serialised by the caller.  Like sph_evaluate it
 * ends a resident state; the context's own buffers are left as they were.
 */
sph_status sph_evaluate_noalloc(sph_ctx *ctx, sph_particles *ps);
int64_t sph_noalloc_max_n(void);

/*
 * Copy a particle set (x, y, z, v, m, u, h) into context-owned device memory
 * for time integration with sph_step.  Evaluates density and forces of the
 * initial state.  Keeps nothing that points into ps.
 */
sph_status sph_upload_state(sph_ctx *ctx, const sph_particles *ps);

/*
 * One kick-drift-kick leapfrog step of the resident state (eqs. EQN:LFKDK1,
 * EQN:LFKDK2; loop order of section 5.1): half kick of v and u, drift of x
 * (wrapped into a periodic box), neighbour search, density, forces at the
 * predicted v* = v + a dt and u* = u + du dt, closing half kick, new CFL
 * step min_i dt_i.  dt > 0 fixes the step; dt <= 0 takes the CFL step of the
 * latest forces (read on the device; no host round trip).  If dt_used is not
 * NULL it receives the step actually taken when sph_sync next returns.
 */
sph_status sph_step(sph_ctx *ctx, double dt, double *dt_used);

/*
 * Hierarchical block time-steps (section 2.1.4) with the predictive and
 * reactive time-step limiter (section 2.1.5), on the resident state of a
 * context created with block_lmax > 0 (then sph_step is SPH_ESTATE).  One
 * level-0 step of length dt_max holds 2^block_lmax ticks; a particle on
 * level l steps 2^(block_lmax - l) ticks.  At sph_upload_state and at every
 * full synchronisation dt_max = min_i dt_i 2^k with k the largest integer
 * keeping dt_max <= max_i dt_i (dt_i the CFL steps), and each particle takes
 * the smallest level l with dt_max 2^-l <= dt_i.  One call advances to the
 * next tick at which some particle's step ends:
 *   every particle drifts with its half-step velocity; every particle is
 *   predicted to that time (v_half + a (t - t_mid)); the particles whose step
 *   ends (active) get h, rho and forces from all neighbours (inactive ones
 *   with their stored h, rho, Omega and predicted v, u) and their closing
 *   kick;  levels of active particles: any deeper level at once, one level
 *   shallower only when the time is a multiple of that step, never more
 *   than block_lim levels shallower than their deepest force neighbour
 *   (predictive limiter); active particles mark inactive force neighbours
 *   more than block_lim levels shallower than themselves, which move to
 *   that level, end their step at its next tick and have their opening kick
 *   corrected to the shortened step (reactive limiter); opening kicks.
 * Everything runs on the device (no waiting).  sph_state_info reports the
 * sub-steps, level-0 steps and the clock; at a synchronisation
 * (block_synchronised = 1) sph_download_state returns every particle at the
 * same time; otherwise positions are current and v, u (and alpha) are
 * those of each particle's last synchronisation.  Viscosity switches follow
 * each particle's own steps: under SPH_AV_MM97 alpha is opened, predicted
 * (every particle's forces see the predicted alpha of its neighbours),
 * closed and corrected by the reactive limiter exactly as u is, its rate
 * taken from each force evaluation of the particle; under SPH_AV_CD10 an
 * active particle's alpha is updated after its forces with dt = its own
 * step length and div v of its previous evaluation.  A per-particle alpha
 * given at upload without a switch stays with its particle.  Many states
 * advance together with sph_batch_substep; no graph capture (SPH_ESTATE).
 */
sph_status sph_substep(sph_ctx *ctx);

/*
 * HIP graph of resident steps.  sph_capture_steps records TWO consecutive
 * sph_step(ctx, dt) calls (same dt semantics; dt <= 0 reads the CFL step on
 * the device at replay time) into a graph held by the context, without
 * executing them; sph_replay_steps launches it on the context's stream (two
 * steps per replay, results bit-for-bit those of two sph_step calls).  The
 * graph holds no memset or copy nodes.  Needs a resident state and a
 * non-null stream; a new upload, a reallocation or sph_set_params drops the
 * graph.
 */
sph_status sph_capture_steps(sph_ctx *ctx, double dt);
sph_status sph_replay_steps(sph_ctx *ctx);

/* Write the resident state back in the caller's original index order:
 * x, y, z, v, u, h and, where non-NULL, rho, omega, pressure, cs, a, dudt,
 * vsig, dt, nngb, nforce (m is constant and not written). */
sph_status sph_download_state(sph_ctx *ctx, sph_particles *ps);

/* Diagnostics of the last sph_forces / sph_upload_state / sph_step
 * (waits for the stream).  SPH_ESTATE before any evaluation. */
sph_status sph_state_info(sph_ctx *ctx, sph_state_stats *info);

/*
 * Meshless finite-volume geometry (section 2.2), for the MFV/MFM schemes:
 *   number density n_i = sum_j W(r_ij, h_i) with h_i = eta n_i^(-1/3)
 *     (eqs. EQN:MFV_NDENS, EQN:MFV_HN; eta from the context's parameters,
 *     about 1 for MFV in 3D) -- the density solve of sph_density with every
 *     mass 1, same Newton-Raphson and stopping rule;
 *   gradient matrix E_i = sum_j (r_j - r_i)(r_j - r_i)^T psi_j(r_i) with
 *     psi_j(r_i) = W(r_ij, h_i) / n_i (eq. EQN:MFVEMATRIX) and B_i = E_i^-1;
 *   least-squares gradients grad f_i = sum_j (f_j - f_i) B_i (r_j - r_i)
 *     psi_j(r_i) (eqs. EQN:MFVGRADIENT, EQN:MFVPSI) of up to 4 fields; where
 *     cond_i = |E_i|_F |B_i|_F / 3 exceeds 100 the SPH estimate
 *     n_i^-1 sum_j (f_j - f_i) grad_i W(r_ij, h_i) is returned instead.
 * All arrays are device arrays in caller order.  h: in the guess, out the
 * solved value.  ndens, nngb, B[k], cond, grad[3 q + a] may be NULL (not
 * written).  B holds xx, xy, xz, yy, yz, zz.  Waits for nothing; errors as
 * for sph_density (SPH_ENOTCONVERGED etc. through sph_sync).
 */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
    double *h;
    double *ndens;            /* n_i */
    int32_t *nngb;            /* neighbours j != i with r_ij < R h_i */
    double *B[6];             /* E^-1: xx, xy, xz, yy, yz, zz */
    double *cond;             /* |E|_F |E^-1|_F / 3 */
    int32_t nfields;          /* 0..4 */
    const double *f[4];       /* fields whose gradients are wanted */
    double *grad[12];         /* d f_q / d x_a at [3 q + a] */
} sph_mfv_set;

sph_status sph_mfv_gradients(sph_ctx *ctx, sph_mfv_set *s);

/*
 * Neighbour lists, for tests and export, at the given h (no h solve):
 *   mode 0: j != i with r_ij^2 < (R h_i)^2        (density neighbours)
 *   mode 1: j != i with r_ij^2 < (R h_i)^2 or r_ij^2 < (R h_j)^2  (force)
 * r_ij^2 is formed exactly as (dx*dx + dy*dy) + dz*dz with the minimum image
 * per axis and no fused multiply-add.  offsets: device int64[n+1], idx:
 * device int32[cap]; the lists of particle i are idx[offsets[i] ..
 * offsets[i+1]) in ascending order of j.  SPH_ECAP if they exceed cap
 * (offsets is still complete).  Waits for the stream.
 */
sph_status sph_neighbours(sph_ctx *ctx, const sph_particles *ps, int32_t mode,
                          int64_t *offsets, int32_t *idx, int64_t cap);

/*
 * Batched evaluation (many independent particle sets of uneven size).  The
 * per-set preparation (sort, tree) is enqueued set by set, then the density
 * (or force) loops of all sets run as ONE persistent kernel launch per group
 * of sets sharing precision and leaf size (up to 128 sets per launch): waves
 * claim leaves across all sets, so small sets fill the GPU together.  Each
 * set's results are bit-for-bit those of the single-set call: the work done
 * for a leaf depends on its own set only.  All contexts must be distinct,
 * on one device and bound to the same stream; ps[r] belongs to ctx[r].
 */
sph_status sph_batch_density(sph_ctx *const *ctx, sph_particles *const *ps, int32_t count);
sph_status sph_batch_forces(sph_ctx *const *ctx, sph_particles *const *ps, int32_t count);
/* sph_evaluate over many sets: the density loops of all sets in one launch
 * per group, then their force loops; each set's results are bit-for-bit
 * those of sph_evaluate on that set alone. */
sph_status sph_batch_evaluate(sph_ctx *const *ctx, sph_particles *const *ps, int32_t count);
/* One sph_step of each resident state, pair loops batched as above. */
sph_status sph_batch_step(sph_ctx *const *ctx, int32_t count, double dt);
/* One sph_substep of each block time-step state (each on its own clock),
 * pair loops batched as above; each set's state afterwards is bit-for-bit
 * that of sph_substep on it alone.  SPH_ESTATE, before anything is
 * enqueued, if a context holds no resident state or has block_lmax = 0. */
sph_status sph_batch_substep(sph_ctx *const *ctx, int32_t count);

/* Wait for the context's stream; return and clear the sticky device status. */
sph_status sph_sync(sph_ctx *ctx);

/* Readable description of the last error on this context ("" if none). */
const char *sph_last_error(const sph_ctx *ctx);

/* Bytes of device memory the context currently holds. */
size_t sph_device_bytes(const sph_ctx *ctx);

/* Bytes of device memory a context needs for n particles with these
 * parameters (what it would allocate; no allocation is made).  For
 * admission control by HBM budget. */
size_t sph_plan_bytes(const sph_params *p, int64_t n);

/*
 * Instrumentation.  enable bit 0: timing of individual kernels with HIP
 * events on the context's stream -- the density-loop and force-loop kernels
 * are bracketed by events; sph_kernel_times (waits for the stream) returns the
 * summed milliseconds and launch counts since the last reset.  which: 0
 * density loop, 1 force loop, 2 neighbour build (keys, sort, gather, tree).
 * enable bit 1: the pair loops also count their particle-box and
 * particle-candidate tests (sph_state_stats *_box_tests, *_candidate_tests;
 * zero otherwise), at a cost of a few percent.  Other bits: SPH_EINVAL.
 */
sph_status sph_enable_kernel_timing(sph_ctx *ctx, int32_t enable);
sph_status sph_kernel_times(sph_ctx *ctx, int32_t which, double *ms, int64_t *launches);

/*
 * Request executor for serving many independent particle sets from host
 * memory.  A server owns `slots` slots on the HIP device that is current
 * at sph_server_create, driven by `threads` native worker threads (slot k by
 * thread k mod threads).  Each slot has one non-blocking HIP stream, one
 * context and device arrays plus pinned host staging, all grown to the
 * largest request the slot has run and kept between requests.  A request
 * handed to an idle slot is carried by the slot's thread:
 *   - its host inputs go to the device in one copy through the staging;
 *   - evaluate: sph_evaluate;
 *   - integrate: sph_upload_state, then steps with the CFL step (dt <= 0)
 *     replayed two at a time from sph_capture_steps (plus one sph_step for
 *     an odd count), then sph_download_state;
 *   - the copies of its outputs back are enqueued, and the thread goes on to
 *     its other slots; once the slot's stream has drained, the outputs are
 *     written into the caller's host arrays and the request is marked done.
 * So one thread keeps several requests in flight while it stages the next.
 * Different slots run concurrently; their kernels overlap on the device.
 * Which request goes to which slot and when (admission under an HBM budget)
 * is the caller's choice: sph_server_plan_bytes gives what a slot holds.
 * Results are bit-for-bit those of the same calls made one by one on a
 * fresh context: the library's results do not depend on what a context
 * ran before.  A request computes nothing of its own: its work is that of
 * the entry points it runs (density and forces of section 2.1.1, the
 * time-step of section 2.1.4, the kick-drift-kick steps of section 2.1.3).
 */
#define SPH_REQUEST_EVALUATE  0
#define SPH_REQUEST_INTEGRATE 1
#define SPH_REQUEST_ERROR_LEN 160

/* FP64 fields of a request, in this order (the first nine are its inputs) */
enum {
    SPH_F_X = 0, SPH_F_Y, SPH_F_Z, SPH_F_VX, SPH_F_VY, SPH_F_VZ, SPH_F_M, SPH_F_U, SPH_F_H,
    SPH_F_RHO, SPH_F_OMEGA, SPH_F_PRESSURE, SPH_F_CS, SPH_F_AX, SPH_F_AY, SPH_F_AZ,
    SPH_F_DUDT, SPH_F_VSIG, SPH_F_DT,
    SPH_NF64,
    SPH_NIN = SPH_F_H + 1
};

typedef struct {
    /* set by the caller */
    int32_t kind;          /* SPH_REQUEST_EVALUATE or SPH_REQUEST_INTEGRATE */
    int32_t nsteps;        /* integrate: number of steps (>= 0); with
                              params.block_lmax > 0, level-0 steps of block
                              time-steps (sph_substep until that many full
                              synchronisations, one sub-step in flight at a
                              time: the slot's thread reads the device clock
                              between them without blocking other slots) */
    sph_params params;     /* method and launch parameters of this request */
    int64_t n;             /* particles (>= 0) */
    const double *in[SPH_NIN]; /* HOST inputs, n values each, all non-NULL: x, y, z,
                              vx, vy, vz, m, u and the guess of h */
    double *out[SPH_NF64]; /* HOST outputs by field (n values each), NULL when not
                              wanted.  evaluate writes h .. dt (the fields
                              sph_evaluate writes, h the solved value); integrate
                              writes every field but m (the state after the last
                              step, as sph_download_state gives it).  Entries a
                              kind does not write are ignored. */
    int32_t *iout[2];      /* HOST outputs nngb, nforce (n each), or NULL */
    /* set by the executor once the request is done */
    int32_t status;        /* sph_status of the request */
    int32_t slot;          /* slot that ran it */
    int64_t interactions;  /* n_dens_pairs + n_force_pairs of the last
                              evaluation, times max(nsteps, 1) for integrate;
                              with block time-steps the pairs of the active
                              particles summed over the sub-steps */
    sph_state_stats info;  /* sph_state_info after the request (zero on error) */
    double host_seconds[4];/* staging the inputs and enqueueing the work (the
                              slot thread's time), then in flight on the device
                              until the thread saw it done, then reading the
                              status and writing the outputs (the thread's time) */
    char error[SPH_REQUEST_ERROR_LEN]; /* readable error ("" when status is SPH_OK) */
} sph_request;

typedef struct sph_server sph_server;

/* `slots` (1..64) slots on the current HIP device, driven by `threads`
 * (1..slots; 0 = one per slot) worker threads, started here.  Nothing is
 * allocated on the device until a slot runs its first request.  *s is NULL
 * on error (SPH_EINVAL for a bad count, SPH_EDEVICE without a device). */
sph_status sph_server_create(sph_server **s, int32_t slots, int32_t threads);

/* Hand request r to slot `slot`, which must be idle (no request submitted
 * and not yet returned by sph_server_wait).  Returns at once.  r and every
 * host array it names stay owned by the caller, who must keep them valid and
 * leave them untouched until sph_server_wait has returned r.  A bad slot, a
 * busy slot or a malformed request (bad kind, n < 0, nsteps < 0, a missing
 * input) returns SPH_EINVAL and queues nothing; errors of
 * the run itself (parameters, memory, the method) come back in r->status and
 * r->error.  A request of n = 0 completes at once with SPH_OK. */
sph_status sph_server_submit(sph_server *s, int32_t slot, sph_request *r);

/* Completed requests, oldest first: stores up to `max` of them in done[] and
 * returns how many (0 when none completed within timeout_s seconds; 0 s
 * polls, a negative timeout waits without limit while any request is
 * running).  A slot is idle again before its request is returned.  Returns
 * -1 for bad arguments. */
int32_t sph_server_wait(sph_server *s, sph_request **done, int32_t max, double timeout_s);

/* Free the context, device arrays and pinned staging of an idle slot (its
 * next request allocates them again).  SPH_EINVAL for a bad or busy slot. */
sph_status sph_server_release(sph_server *s, int32_t slot);

/* Device bytes slot `slot` holds now (context plus particle arrays);
 * 0 for a bad slot. */
size_t sph_server_slot_bytes(sph_server *s, int32_t slot);

/* Device bytes a slot needs to run a request of n particles with parameters
 * p: sph_plan_bytes plus the request's particle arrays (19 FP64 and 2 int32
 * values per particle).  No allocation is made. */
size_t sph_server_plan_bytes(const sph_params *p, int64_t n);

/* Wait for the running requests, stop the threads and free everything the
 * server owns.  Requests still unreturned by sph_server_wait are complete
 * when it returns.  NULL is a no-op. */
sph_status sph_server_destroy(sph_server *s);

#ifdef __cplusplus
}
#endif

#endif /* SPH_MI355X_H */
