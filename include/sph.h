/*
 * sph.h -- C interface of the MI355X (gfx950) SPH neighbour-interaction sweep.
 *
 * The sweep is the per-step hot path of the tree-SPH method of "Smoothed
 * Particle Hydrodynamics in pkdgrav3 for Shock Physics Simulations. I.
 * Hydrodynamics" (Meier, Potter, Reinhardt, Stadel):
 *   tree build over particle buckets          (Sec. 2.1 reordered storage, Sec. 2.3.2 bounds)
 *   bucket neighbour search by bound overlap  (Sec. 2.3.2, Fig. 1)
 *   density sum + smoothing-length iteration (Sec. 2.3.3, eq:Density_estimate)
 *   force loop, du/dt, viscosity, time step  (Sec. 2.3.5, eq:AV_heating; Sec. 2.3.6, eq:courant_condition)
 *   kick-drift-kick with predictor            (Sec. 2.3.6)
 *
 * Conventions
 *   H        kernel support radius (W = 0 for r >= H); h = H/2 is the smoothing
 *            length that enters the viscosity and the Courant limit.
 *   x_ij     x_i - x_j, minimum image per component in a periodic box.
 *   G_i      gather set {j != i : r_ij^2 < H_i^2}; the density includes i.
 *   F_i      force set  {j != i : r_ij^2 < max(H_i, H_j)^2}.
 *
 * Memory and ownership
 *   Every particle array in sph_particles is a caller-owned DEVICE pointer to
 *   n contiguous doubles in the caller's particle order (structure of arrays).
 *   The caller keeps them alive until the work enqueued on the stream has
 *   completed.  The context owns everything else (sorted copies, tree, walk
 *   stacks, counters; about 280 bytes per particle at buckets of 32, 320 in
 *   mixed precision) and reuses it: after the first call at a given n no
 *   further device allocation happens, so the step can be captured into a
 *   HIP graph.
 *   A context is not thread-safe; use one context per stream.
 *
 * Streams
 *   `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   work is enqueued asynchronously; no call synchronises the host except
 *   sph_neighbors (it returns the needed size), sph_get_stats and
 *   sph_autotune.
 *
 * Errors
 *   Argument errors return SPH_ERR_INVALID synchronously and enqueue nothing.
 *   HIP runtime errors return SPH_ERR_HIP.  Conditions found on the device go
 *   to a device status word, cleared at the start of every call:
 *     SPH_ERR_NOCONV     a smoothing-length iteration stopped at nr_maxit;
 *     SPH_ERR_NONFINITE  a non-finite H, rho, Omega, a, du/dt or dt.
 *   The status of a call is surfaced (1) by sph_get_stats (sph_stats.status,
 *   with the counts), which synchronises, and (2) by the NEXT call on the
 *   context once the device has finished the call that set it: that next call
 *   then returns the status and enqueues nothing (the status is reported
 *   once; calling again proceeds).  A call never waits for the device to
 *   learn the status.  Conditions that are not errors (H held at the cap
 *   h_max, a walk that fell back to the linear bucket test) are counted in
 *   sph_stats only.  sph_last_error() gives a text for the last failing call.
 *   No C++ exception crosses this interface.
 */
#ifndef SPH_MI355X_H
#define SPH_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sph_ctx sph_ctx;

typedef enum {
    SPH_OK = 0,
    SPH_ERR_INVALID = 1,  /* bad argument, shape or parameter */
    SPH_ERR_OOM = 2,      /* device allocation failed */
    SPH_ERR_HIP = 3,      /* HIP runtime error */
    SPH_ERR_CAPACITY = 4, /* output buffer too small (see sph_neighbors) */
    SPH_ERR_NOCONV = 5,   /* the smoothing-length iteration of some particle reached
                             nr_maxit without converging (device status word) */
    SPH_ERR_STATE = 6,    /* call out of order (e.g. density before a tree) */
    SPH_ERR_NONFINITE = 7 /* a NaN or infinity in H, rho, Omega, a, du/dt or dt
                             (device status word) */
} sph_status;

enum { SPH_KERNEL_M4 = 0, SPH_KERNEL_WC2 = 1, SPH_KERNEL_WC4 = 2, SPH_KERNEL_WC6 = 3 };
enum { SPH_PREC_FP64 = 0, SPH_PREC_MIXED = 1 };
enum { SPH_EOS_IDEAL = 0, SPH_EOS_STIFFENED = 1 };
enum { SPH_MODE_GATHER = 0, SPH_MODE_FORCE = 1 };

/* Method parameters.  sph_default_params() fills the defaults noted here. */
typedef struct {
    int32_t kernel;    /* SPH_KERNEL_*: cubic spline (Monaghan 1992) or Wendland C2/C4/C6
                          (Dehnen & Aly 2012), Sec. 2.3.  Default M4. */
    int32_t precision; /* SPH_PREC_FP64: all pair arithmetic in FP64.
                          SPH_PREC_MIXED: pair arithmetic in FP32 on coordinates
                          relative to the sink group, the pair terms summed in FP64;
                          positions, the step and the global reductions stay FP64.
                          Default FP64. */
    int32_t eos;       /* SPH_EOS_IDEAL: P = (gamma-1) rho u (Sec. 2.3.1).
                          SPH_EOS_STIFFENED: P = (gamma-1) rho u - gamma P0. */
    int32_t periodic;  /* 1: periodic box [box_lo, box_hi) with minimum image;
                          0: open boundary (box ignored).  Default 1. */
    double n_ngb;      /* target neighbour number of the constant kernel mass rule
                          (4 pi/3) H^3 rho = n_ngb m_i (Sec. 2.3.3).  Must exceed
                          (4 pi/3) sigma of the kernel.  Default 64. */
    double box_lo[3], box_hi[3]; /* periodic box.  Default unit cube. */
    double gamma, P0;  /* EOS constants.  Default 5/3, 0. */
    double alpha, beta, eps_av; /* Monaghan viscosity (Sec. 2.3.5).  Default 1, 2, 0.01. */
    double eta_c, eta_a, dt_max; /* Courant factor, acceleration factor (Sec. 2.3.6),
                                    cap on the step.  Default 0.3, 0.2, 1. */
    double h_max;      /* cap on H (also kept below half the periodic box).  Default 0.25. */
    double oversel;    /* the density pass searches with oversel*H so the iteration can
                          grow H without a new walk (Sec. 2.3.3).  Default 1.1. */
    double nr_tol;     /* relative tolerance on the Newton step of H.  Default (when 0)
                          1e-14 for FP64, 1e-5 for mixed.  A Halley step below
                          sqrt(tol) H (FP64) or 2e-3 H (mixed) is taken without
                          another scan, with rho and Omega Taylor-corrected. */
    int32_t nr_maxit;  /* iteration cap.  Default 64. */
    int32_t bucket;    /* particles per bucket: 8, 16, 32 or 64; 0 = autotuned.  Default 32. */
    int32_t stack_limit; /* entries of the per-wavefront walk stack in use, 2..768 (0 = 768).
                            A walk that would outgrow it restarts as a test of every bucket
                            of the set; results do not change, only the cost. */
    int32_t flags;     /* SPH_FLAG_* (0 = the plain scheme):
                          SPH_FLAG_ENTROPY: entropy-conserving update of u (Sec. 2.3.5):
                            du/dt holds only the viscous heating (eq:AV_heating); after
                            each step's density pass u is carried along the adiabat from
                            the previous density to the new one, u(rho_new, s(rho_old,
                            u_old)), for the ideal gas (P/rho^gamma fixed) and the stiffened
                            gas ((P + P0)/rho^gamma fixed).
                          SPH_FLAG_EVOLVED: evolved density (Sec. 2.3.3): rho is a state
                            variable kicked and predicted like u with the continuity rate
                            d rho_i/dt = (1/Omega_i) sum m_j (v_ij . x_ij) G_i from the force
                            pass (written to drhodt); the density pass still sets H and
                            Omega.  Not combined with SPH_FLAG_ENTROPY.
                          SPH_FLAG_INTERFACE: interface correction (Sec. 2.3.4) before
                            every force pass: the kernel imbalance
                            I_i = ic_alpha |sum_j kappa_ij (x_j - x_i) m_j W_ij(h_i)|
                                  / (h_i sum_j m_j W_ij(h_i))  (eq:Kernel_imbalance;
                            kappa = +1 within a material, -1 across, h = H/2, the sums
                            over G_i and i), averages Tbar, Pbar of T = u and P with
                            weights exp(-I_j^2) W_ij(h_i), the corrected P~ and T~ and
                            rho~ = rho_EOS(T~, P~); the force pass uses rho~, P~ and the
                            sound speed at (rho~, T~).  Not combined with SPH_FLAG_EVOLVED.
                          SPH_FLAG_DYNAMIC: dynamic per-region bucket sizing (Sec. 2.3.2,
                            last paragraph): the tree is built over buckets of 8 and each
                            sink group walks it down to its own bucket size 8, 16, 32 or
                            64, starting from `bucket` and adjusted every force pass from
                            the group's interaction-list length (candidate particles per
                            neighbour pair): long lists halve the buckets, short ones
                            double them.  The level is carried by the particles from step
                            to step.  Results do not depend on it, only the cost.
                          SPH_FLAG_RUNGS: individual time steps (Sec. 2.3.6): particle i
                            steps with dt_max 2^-r_i, its rung r_i in 0..rung_max the
                            smallest with min(dt_a, dt_CFL) >= dt_max 2^-r_i, raised so
                            that r_i >= r_j - 2 for every j of F_i (Saitoh-Makino; the
                            neighbours' rungs before the update), moved to a longer step
                            only at a boundary of that step.  sph_init assigns the rungs
                            (the limiter against the neighbours' desired rungs); each
                            sph_step is then one substep: opening kick of the particles
                            at a step boundary, drift of all to the next boundary of any
                            particle, density, prediction of v and u at that time
                            (v_half + (t - t_mid) a for a step whose middle is t_mid),
                            EOS, forces of the particles whose step ends there (the
                            active ones), their closing kick and new rung.  With fastgas
                            > 0 and fewer than fastgas n active particles, the density
                            pass runs only for the particles on the interaction lists of
                            the active ones (FastGas, Sec. 2.3.6, last paragraph: lists
                            taken with the sinks' H widened by oversel).  Single-set
                            contexts only; not combined with the other flags. */
    double ic_alpha;   /* normalisation alpha of the kernel imbalance (the paper gives no
                          value).  Default 10 (I near 1.5 at the free surface of a
                          uniform body). */
    int32_t rung_max;  /* SPH_FLAG_RUNGS: finest rung, 0..20 (time is counted in units of
                          dt_max 2^-rung_max).  Default 8. */
    int32_t launch;    /* launch shape of the density and force sweeps.  The first two
                          take each sink group's interaction list from a walk kernel
                          run before the sweep (stored in the context, up to 4096
                          buckets per group; a longer list, or in the density pass a
                          root beyond the stored list's radius, sends the group to a
                          sweep kernel that walks the tree itself):
                          SPH_LAUNCH_GROUPS: one workgroup (one wavefront) per sink group;
                          SPH_LAUNCH_PERSISTENT: as many workgroups as the GPU holds at
                            once, each taking sink groups from per-XCD queues until none
                            is left (each XCD's queue is one contiguous run of groups; an
                            XCD that runs dry takes from the next);
                          SPH_LAUNCH_WALK: one workgroup per sink group, each walking the
                            tree itself (no stored lists).
                          Results do not depend on it, only the cost; sph_autotune picks
                          one.  SPH_FLAG_RUNGS takes SPH_LAUNCH_GROUPS or SPH_LAUNCH_WALK
                          (its substeps sweep the groups of the sink lists);
                          sph_init_noalloc walks in the sweep kernels.
                          Default SPH_LAUNCH_GROUPS. */
    double fastgas;    /* SPH_FLAG_RUNGS: active fraction below which the density pass is
                          restricted (0 = never).  Default 0. */
} sph_params;

enum { SPH_LAUNCH_GROUPS = 0, SPH_LAUNCH_PERSISTENT = 1, SPH_LAUNCH_WALK = 2 };

enum {
    SPH_FLAG_ENTROPY = 1, SPH_FLAG_EVOLVED = 2, SPH_FLAG_INTERFACE = 4, SPH_FLAG_DYNAMIC = 8,
    SPH_FLAG_RUNGS = 16
};

/* Caller-owned device arrays, n doubles each, caller particle order.
 * State: x y z (positions inside the periodic box), vx vy vz, m, u, H (and
 * rho with SPH_FLAG_EVOLVED).
 * Results written by the calls: rho, omega (grad-h term), P, c (pressure and
 * sound speed), ax ay az, dudt, dt (per-particle time-step limit), drhodt
 * (continuity rate; only with SPH_FLAG_EVOLVED, may be NULL otherwise).
 * Interface correction (SPH_FLAG_INTERFACE): mat holds each particle's
 * material id (integer values; NULL = one material); imb and rhoc receive the
 * kernel imbalance and the corrected density (each may be NULL).
 * Individual time steps (SPH_FLAG_RUNGS): rung holds each particle's rung
 * (integer values, written by sph_init and the steps).  Between substeps a
 * particle at a step boundary holds v and u at the current time, the others
 * their half-step values; ax, ay, az, dudt and dt are those of each
 * particle's last force pass. */
typedef struct {
    double *x, *y, *z, *vx, *vy, *vz, *m, *u, *H;
    double *rho, *omega, *P, *c, *ax, *ay, *az, *dudt, *dt;
    double *drhodt;
    double *mat, *imb, *rhoc;
    double *rung;
} sph_particles;

/* Counters of the most recent call, read with sph_get_stats. */
typedef struct {
    int64_t n;                    /* particles */
    int64_t pairs_density;        /* sum_i |G_i| at the H of the last scan of the candidates;
                                     the iteration may then take a last step of at most
                                     sqrt(nr_tol) H (FP64) or 2e-3 H (mixed) without another
                                     scan, so a pair within that distance of the final support
                                     may be counted on the other side (at 2M particles, FP64:
                                     within 1e-7 of the oracle's count at its H) */
    int64_t pairs_force;          /* sum_i |F_i| */
    int64_t cand_density;         /* candidate particles tested, summed over sinks and scans */
    int64_t cand_force;           /* candidate particles tested in the force pass */
    int64_t nr_iter_max;          /* largest number of density scans in a sink group */
    int64_t nr_scans;             /* density scans summed over sink groups */
    int64_t n_noconv;             /* particles whose H hit the cap or the iteration limit */
    int64_t n_rewalk;             /* sink groups re-walked because H outgrew the search radius */
    int64_t n_overflow;           /* sink groups whose tree walk outgrew its stack and fell
                                     back to testing every bucket (results stay exact) */
    double momentum[3];           /* sum m v after the last step (FP64) */
    double e_kin, e_int;          /* sum m v^2/2, sum m u after the last step (FP64) */
    double dt_next;               /* min_i dt_i from the last force pass, capped by dt_max */
    double dt_used;               /* step size of the last sph_step */
    int64_t pairs_density_total;  /* running sums of pairs_density / pairs_force over */
    int64_t pairs_force_total;    /* every call since the context was created */
    double t_tree_ms;             /* with sph_set_timing on: device time of the last call's */
    double t_density_ms;          /* tree build, density kernel, force kernel and the whole */
    double t_forces_ms;           /* call (HIP events on the call's stream); -1 when the */
    double t_total_ms;            /* phase did not run or timing is off */
    int64_t n_iter_limit;         /* particles whose iteration stopped at nr_maxit */
    int64_t n_nonfinite;          /* particles with a non-finite output */
    int64_t n_retest;             /* mixed path: pairs near a neighbour-set boundary whose
                                     membership was decided by an FP64 re-test */
    int32_t status;               /* device status word of the last call: SPH_OK,
                                     SPH_ERR_NOCONV or SPH_ERR_NONFINITE */
    int32_t reserved_;
    int64_t slots_density;        /* candidate particles loaded from the interaction lists */
    int64_t slots_force;          /* (before the per-particle filter), per pass */
    int64_t groups_by_level[4];   /* force-pass sink groups with buckets of 8, 16, 32, 64
                                     (SPH_FLAG_DYNAMIC; else all in the tree's size) */
    int64_t t_units;              /* SPH_FLAG_RUNGS: time after the last call, in units of
                                     dt_max 2^-rung_max (dt_used is the substep's length) */
    int64_t n_active;             /* particles whose force was computed by the last call */
    int64_t n_dens;               /* particles whose density was computed by the last call */
    int64_t n_fastgas_miss;       /* force-set neighbours of active particles that FastGas
                                     left out of the density pass (their density is that
                                     of an earlier substep) */
    int64_t launch;               /* SPH_LAUNCH_* of the last call's sweeps */
    int64_t workgroups_force;     /* workgroups of the last force launch (sink groups, or
                                     the resident grid of a persistent launch) */
    double t_force_walk_ms;       /* with timing on: device time of the force pass's and */
    double t_density_walk_ms;     /* the density pass's tree walks (kernels of their own,
                                     before the sweep kernels, whose times are t_forces_ms
                                     and t_density_ms); -1 when they did not run */
    int64_t groups_walked;        /* sink groups of the last call whose interaction list
                                     was too long to store (or, in the density pass, whose
                                     root lay beyond the stored list): swept again from the
                                     start by the kernel that walks the tree itself */
} sph_stats;

/* Fills *p with the defaults listed above. */
void sph_default_params(sph_params *p);

/* Library version text (static storage). */
const char *sph_version(void);

/* Text of the last error on this context (static storage owned by ctx). */
const char *sph_last_error(const sph_ctx *ctx);

/* Creates a context for one particle set.  Allocates nothing on the device
 * until the first sph_build_tree.  Returns SPH_ERR_INVALID on bad params. */
sph_status sph_create(const sph_params *params, sph_ctx **out);

/* Creates a context for `nsets` independent particle sets processed together
 * (one tree per set, all sets in the same launches).  set_offsets: host array
 * of nsets+1 increasing int64; set s owns particles [set_offsets[s],
 * set_offsets[s+1]) of every particle array.  set_box: host array of
 * 6*nsets doubles (lo x y z, hi x y z per set) or NULL for params->box_*.
 * nsets <= 4096. */
sph_status sph_create_batch(const sph_params *params, int32_t nsets, const int64_t *set_offsets,
                            const double *set_box, sph_ctx **out);

/* Frees the context and all device memory it owns (synchronises the device). */
void sph_destroy(sph_ctx *ctx);

/* Tree build (Sec. 2.1, Sec. 2.3.2): Hilbert keys of x y z within the box,
 * stable radix sort, gather into sorted order, buckets of `bucket` particles,
 * cell bounds, box-of-balls and ball-of-balls from H, combined bottom-up over
 * a binary tree of buckets.  Reads x y z m H.  n must equal the set total for
 * batch contexts. */
sph_status sph_build_tree(sph_ctx *ctx, const sph_particles *p, int64_t n, void *stream);

/* Neighbour sets of the current tree and H (Sec. 2.3.2).  mode SPH_MODE_GATHER
 * gives G_i, SPH_MODE_FORCE gives F_i.  Output in CSR form on the device:
 * offsets (n+1 int64, row of caller particle i = [offsets[i], offsets[i+1]))
 * and idx (int32 caller indices; in a batch context, indices into the whole
 * concatenated particle arrays), each row ascending, self excluded.  If capacity < total the call writes offsets only, sets
 * *needed (host) and returns SPH_ERR_CAPACITY; call again with a larger idx.
 * Synchronises the stream.  Rows longer than 4096 return SPH_ERR_CAPACITY. */
sph_status sph_neighbors(sph_ctx *ctx, const sph_particles *p, int32_t mode, int64_t *offsets,
                         int32_t *idx, int64_t capacity, int64_t *needed, void *stream);

/* Density pass (Sec. 2.3.3) on the current tree: per particle, H solving
 * (4 pi/3) H^3 rho(H) = n_ngb m_i by a bracket-safeguarded Halley iteration
 * (Newton with the second derivative of the same sums) on the over-selected
 * candidate list, rho = sum_{G_i + i} m_j W(r_ij, H_i), and
 * Omega = 1 + (H/(3 rho)) d rho/dH.  Reads H as the first guess; writes H,
 * rho, omega; refits the ball bounds of the tree with the new H. */
sph_status sph_density(sph_ctx *ctx, sph_particles *p, void *stream);

/* Force pass (Sec. 2.3.5, 2.3.6) on the current tree and H: EOS from rho and
 * u (written to P, c; with SPH_FLAG_INTERFACE the corrected values of Sec.
 * 2.3.4), then a, du/dt (pressure + viscosity) and the per-particle limit
 * dt = min(eta_a sqrt(H/|a|), Courant limit, dt_max).  Uses v and u as given. */
sph_status sph_forces(sph_ctx *ctx, sph_particles *p, void *stream);

/* Start-up: sph_build_tree(n) + density + forces at the initial time, and the
 * reductions (so sph_step can take its first dt from the device). */
sph_status sph_init(sph_ctx *ctx, sph_particles *p, int64_t n, void *stream);

/* One kick-drift-kick step (Sec. 2.3.6) with global step dt (dt <= 0: the
 * minimum per-particle limit of the previous force pass, read on the device):
 * opening kick, drift with periodic wrap, tree build, density, predictor,
 * EOS, forces with the predicted v and u, closing kick, FP64 reductions.
 * With SPH_FLAG_ENTROPY the half-step u moves along the adiabat to the new
 * density right after the density pass (and the prediction of u with it);
 * with SPH_FLAG_EVOLVED rho is kicked and predicted like u and the density
 * pass leaves it untouched.  Requires a previous sph_init or sph_step. */
sph_status sph_step(sph_ctx *ctx, sph_particles *p, double dt, void *stream);

/* Captures one sph_step (same arguments) into a HIP graph owned by the
 * context and launches nothing.  sph_graph_launch replays it on `stream`. */
sph_status sph_graph_capture_step(sph_ctx *ctx, sph_particles *p, double dt, void *stream);
sph_status sph_graph_launch(sph_ctx *ctx, void *stream);

/* Picks the bucket size (8, 16, 32, 64) and the sweeps' launch shape
 * (SPH_LAUNCH_*; SPH_LAUNCH_GROUPS only with SPH_FLAG_RUNGS) for the given
 * particles.  Every combination runs sph_init from the same first guess of H,
 * then a density and a force pass from the converged H.  Those two passes are
 * timed, walk kernels included; with SPH_FLAG_RUNGS, sph_init's own passes
 * are.  Synchronises.  Leaves H, rho, omega, P, c, a, dudt, dt as sph_init
 * writes them.  The choice is kept in the context; the bucket size comes
 * back in *bucket and the launch shape in sph_stats.launch. */
sph_status sph_autotune(sph_ctx *ctx, sph_particles *p, int32_t *bucket, void *stream);

/* Turns device-side phase timing on (1) or off (0); timings appear in sph_stats.
 * Timing is skipped inside graph capture. */
sph_status sph_set_timing(sph_ctx *ctx, int32_t enable);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the start-up
 * pass of sph_init (tree build, density with the smoothing-length iteration,
 * forces) for one particle set of n <= 65536 particles, with no context and
 * no device or pinned allocation.  Every work array is carved out of one
 * static 32 MiB device array that each GPU the library runs on holds until
 * the process ends.  Reads x y z vx vy vz m u H (H = first guess); writes H,
 * rho, omega, P, c, ax ay az, dudt, dt, equal to what sph_init writes for
 * the same parameters and particles.  Enqueued on `stream`; no counters or
 * status word are kept.  All calls on one GPU share the static array: calls
 * that overlap on one GPU (other streams, other threads) race.  Returns
 * SPH_ERR_CAPACITY for n > 65536 and SPH_ERR_INVALID for bad parameters or
 * NULL arrays, enqueueing nothing. */
sph_status sph_init_noalloc(const sph_params *params, sph_particles *p, int64_t n, void *stream);

/* Synchronises the context's last stream and copies the counters and the
 * status word of the last call (which is then not reported again by the next
 * call).  Returns SPH_OK whenever the copy succeeds. */
sph_status sph_get_stats(sph_ctx *ctx, sph_stats *out);

#ifdef __cplusplus
}
#endif
#endif /* SPH_MI355X_H */
