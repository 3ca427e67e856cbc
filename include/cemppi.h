/*
 * cemppi.h -- C ABI of the MI355X CE-MPPI replan library (libcemppi.so).
 *
 * One call of ce_mppi_replan runs one iteration of clustering-embedded MPPI
 * (Liu, Chang, Chen, "Clustering-Embedded Model Predictive Path Integral
 * Control", Alg. 1) for one planner on the GPU:
 *   noise -> rollouts with cost and collision -> pruning -> reference point
 *   and features -> DBSCAN -> cluster selection -> within-cluster update ->
 *   shift.
 *
 * Conventions (all entry points):
 *  - Every call returns a ce_status; no C++ exception crosses the ABI.  The
 *    text of the last error of the calling thread is available from
 *    ce_mppi_last_error().
 *  - Pointers documented as "device" must point to device memory of the
 *    planner's GPU (e.g. a torch tensor's data_ptr()); "host" pointers to
 *    host memory.  The caller owns every buffer it passes in.
 *  - Arrays are dense, row-major, single precision unless stated.
 *  - Work is enqueued on the HIP stream passed as `stream` (a hipStream_t; 0
 *    is the null stream) and is asynchronous: outputs are valid once that
 *    stream has been synchronised.
 *  - A planner owns its device state (nominal control sequence, obstacle
 *    history, step counter, scratch), all allocated in ce_mppi_create.
 *    ce_mppi_replan allocates nothing.  A planner must not have two calls in
 *    flight on different streams at once (ce_mppi_replan and
 *    ce_mppi_replan_from_rollouts return CE_EBUSY when they can see it);
 *    different planners are independent.
 */
#ifndef CEMPPI_H
#define CEMPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CE_MPPI_ABI_VERSION 1u
#define CE_MPPI_MAX_CTRL 6        /* m                                          */
#define CE_MPPI_MAX_OBSTACLES 64  /* n_obs per planner                          */
#define CE_MPPI_MAX_HORIZON 63    /* N: the N+1 states of a rollout share a wave */
#define CE_MPPI_MAX_HISTORY 16    /* H                                          */
#define CE_MPPI_MAX_SAMPLES 65536 /* K                                          */
#define CE_MPPI_MAX_BATCH 1024    /* planners per batch                         */
#define CE_MPPI_MAX_SPHERES 16    /* arm link spheres                           */

typedef int32_t ce_status;
enum {
  CE_OK = 0,
  CE_EINVAL = 1,       /* invalid argument or configuration                    */
  CE_ENOMEM = 2,       /* device allocation failed                             */
  CE_EDEVICE = 3,      /* HIP runtime error or no usable GPU                   */
  CE_EUNSUPPORTED = 4, /* valid request the library does not support           */
  CE_EBUSY = 5         /* resource in use (e.g. server full)                   */
};

/* f(.) of Sec. II-A: the differential-drive robot of Sec. III-A (state
 * (x, y, theta), control (v, omega), task space (x, y)) and a six-joint serial
 * arm driven by joint velocities as in Sec. III-C (state (q, qdot) in R^12,
 * control qdot command in R^6, task space = end-effector position). */
enum { CE_DYN_UNICYCLE = 0, CE_DYN_ARM6 = 1 };
/* selection rule of Alg. 1: minimum mean cost (static) or most opposite to
 * the estimated obstacle motion (dynamic), Sec. II-B.3 */
enum { CE_SCENE_STATIC = 0, CE_SCENE_DYNAMIC = 1 };
/* point averaged into the collision-derived reference point, Sec. II-B.2:
 * terminal position (the paper's Eq. (11)) or first-contact position */
enum { CE_REF_TERMINAL = 0, CE_REF_FIRST_CONTACT = 1 };

/* ce_mppi_config.flags: optional variants of the rollout model.
 *
 * CE_FLAG_POSE_COST (arm only): the goal-reaching cost of the real-robot
 *   experiment, Sec. III-C.  Stage state x_j (j = 0..N-1) costs
 *     Q[0] |p_ee - p_g| + Q[1] d_R(R_ee, R_g) + Q[2] I_col(x_j)
 *   and the terminal state the same terms with Qf[0..2]; the R control term
 *   and the joint-limit penalty are kept.  p_g = goal[0..2]; R_g is the
 *   rotation vector goal[3..5] (axis times angle, radians); d_R is the angle
 *   of the relative rotation R_g^T R_ee, in [0, pi].  I_col is the contact
 *   of any link sphere with any obstacle; x_0 counts in the cost but, as in
 *   the default model, only x_1..x_N decide the pruning of Eq. (9).  The
 *   paper's weights are (w_p, w_R, w_c) = (10, 3, 1000).
 * CE_FLAG_OBS_CONST_VEL: inside the rollouts every obstacle moves with its
 *   own constant velocity, estimated from the planner's observation history
 *   as in Eq. (17) (zero until two observations with the same obstacle count
 *   exist); state x_j is tested against the obstacles at time j dt.  Needs
 *   history_len >= 2.  Without it the obstacles stay where observed.
 * Unknown bits are rejected with CE_EINVAL. */
#define CE_FLAG_POSE_COST 1u
#define CE_FLAG_OBS_CONST_VEL 2u
/* branch of Alg. 1 taken by a replan */
enum { CE_BRANCH_CLUSTER = 0, CE_BRANCH_FALLBACK = 1, CE_BRANCH_ALL_COLLIDE = 2 };

/* ce_mppi_info.status bits (data-dependent conditions, not errors) */
#define CE_STATUS_FALLBACK 1u    /* no colliding rollout: plain MPPI over all K      */
#define CE_STATUS_ALL_COLLIDE 2u /* every rollout collides: plain MPPI over all K    */
#define CE_STATUS_NO_CLUSTER 4u  /* DBSCAN found no cluster: update over all of V    */
#define CE_STATUS_DYN_STATIC 8u  /* dynamic rule impossible (H'<2 or slow obstacle)  */
#define CE_STATUS_NONFINITE 16u  /* non-finite x_t or obstacle: replan was a no-op   */

/* Planner configuration: the "Require" line of Alg. 1.  Fill with
 * ce_mppi_config_init() and override fields. */
typedef struct ce_mppi_config {
  uint32_t abi_version;      /* CE_MPPI_ABI_VERSION                                     */
  int32_t dynamics;          /* CE_DYN_*                                                */
  int32_t horizon;           /* N, 1..CE_MPPI_MAX_HORIZON                               */
  int32_t num_samples;       /* K, 1..CE_MPPI_MAX_SAMPLES                               */
  float dt;                  /* integration step and observation interval (> 0)        */
  float lambda;              /* temperature of Eq. (6) / Eq. (19), > 0                  */
  float noise_chol[36];      /* L, m x m row-major lower triangular, Sigma = L L^T      */
  float u_min[6], u_max[6];  /* control bounds; -INF/+INF disable the clamp             */
  float dbscan_eps;          /* DBSCAN radius (closed ball), > 0                        */
  int32_t dbscan_min_pts;    /* DBSCAN minPts, the point itself included, >= 1          */
  float norm_eps;            /* epsilon of the normalisations of Eq. (13),(15)-(17)     */
  int32_t scene_mode;        /* CE_SCENE_*                                              */
  int32_t history_len;       /* H of Eq. (17), 1..CE_MPPI_MAX_HISTORY (>=2 if dynamic)  */
  float v_obs_min;           /* obstacle speed below which the static rule is used      */
  int32_t ref_mode;          /* CE_REF_*                                                */
  int32_t max_obstacles;     /* capacity, 0..CE_MPPI_MAX_OBSTACLES                      */
  float robot_radius;        /* unicycle body radius (0 = point robot)                  */
  float goal[6];             /* unicycle: goal state x_f; arm: end-effector target p_g
                                (pose cost: goal[3..5] = goal orientation, rotation vector) */
  float Q[6];                /* unicycle: diag state weight; arm: Q[0] = position weight
                                (pose cost: Q[0..2] = w_p, w_R, w_c)                    */
  float R[6];                /* diag control weight                                     */
  float Qf[6];               /* unicycle: diag terminal weight; arm: Qf[0]              */
  float dh[6][4];            /* arm: per joint (a, d, alpha, theta offset), standard DH */
  int32_t n_link_spheres;    /* arm: collision spheres along the link chain, <= 16      */
  float link_sphere_radius;  /* arm                                                     */
  float q_limit[6];          /* arm: joint-limit penalty threshold |q_i|                */
  float w_limit;             /* arm: joint-limit penalty weight                         */
  uint64_t seed;             /* Philox key                                              */
  uint32_t stream_id;        /* Philox counter word 3 (e.g. the planner id)             */
  int32_t device;            /* HIP device ordinal                                      */
  uint32_t flags;            /* CE_FLAG_* bits, 0 = the default model                   */
} ce_mppi_config;

/* Per-replan diagnostics, written on the device. */
typedef struct ce_mppi_info {
  int32_t branch;          /* CE_BRANCH_*                                     */
  int32_t n_collide;       /* |C^col|                                         */
  int32_t n_feasible;      /* |V|                                             */
  int32_t n_ref;           /* rollouts averaged into the reference point      */
  int32_t n_clusters;      /* M                                               */
  int32_t selected;        /* c*, -1 if none                                  */
  int32_t selected_size;   /* |C_{c*}|                                        */
  int32_t closest;         /* o*, -1 without obstacles                        */
  int32_t rule;            /* CE_SCENE_* actually applied                     */
  int32_t history_used;    /* H' = min(H, observations available)            */
  uint32_t status;         /* CE_STATUS_* bits                                */
  uint32_t step;           /* Philox step word used by this replan           */
  float margin;            /* second-best minus best selection key (INF if M<2) */
  float s_min;             /* minimum cost over the update set                */
  float ref_point[3];      /* collision-derived reference point              */
  float v_obs[3];          /* obstacle velocity estimate, Eq. (17)           */
  float v_obs_hat[3];      /* normalised                                     */
  float weight_sum;        /* sum of exp(-(S - s_min)/lambda) over the set   */
} ce_mppi_info;

typedef struct ce_mppi_planner ce_mppi_planner;

/* Fill *cfg with defaults for the given dynamics (the unit-sized unicycle or
 * arm problem, static rule, no obstacles).  Returns CE_EINVAL for an unknown
 * dynamics or a NULL cfg. */
ce_status ce_mppi_config_init(ce_mppi_config* cfg, int32_t dynamics);

/* Validate *cfg and create a planner on cfg->device: allocates every device
 * buffer, sets the nominal sequence U to zero, empties the obstacle history
 * and sets the step counter to 0.  Errors: CE_EINVAL (bad config; see the
 * limits above), CE_ENOMEM, CE_EDEVICE. */
ce_status ce_mppi_create(const ce_mppi_config* cfg, ce_mppi_planner** out);

/* One replan, Alg. 1.
 *   x_t       device, [n] current state (n = 3 unicycle, 12 arm)
 *   obstacles device, [n_obs][p+1] rows (centre..., radius), p = 2 or 3;
 *             may be NULL when n_obs == 0.  Their centres are pushed into the
 *             planner's history (the {o_{t-h}} of Eq. (17)); a change of n_obs
 *             empties the history first.
 *   u_out     device, [m] control to apply (u_t after the update)
 *   U_out     device, [N][m] updated sequence before the shift, or NULL
 *   info      device, one ce_mppi_info, or NULL
 * The planner keeps the shifted warm start (last control repeated) and
 * increments its step counter.  A non-finite x_t or obstacle value makes the
 * call a no-op apart from u_out = U[0] and info.status.  A planner has at most
 * one replan in flight: a call on a stream other than the planner's previous
 * replan (single or batched) while that stream still has work queued returns
 * CE_EBUSY without enqueuing anything; synchronise that stream first.
 * Errors: CE_EINVAL (NULL planner/x_t/u_out, n_obs outside 0..max_obstacles),
 * CE_EBUSY, CE_EDEVICE. */
ce_status ce_mppi_replan(ce_mppi_planner* planner, const float* x_t, const float* obstacles,
                         int32_t n_obs, float* u_out, float* U_out, ce_mppi_info* info,
                         void* stream);

/* Release every resource of the planner.  NULL-safe.  The caller must have
 * synchronised the streams the planner was used on. */
void ce_mppi_destroy(ce_mppi_planner* planner);

/* ---- planner state ---- */

/* Copy U ([N][m], device) into / out of the planner (asynchronous on stream). */
ce_status ce_mppi_set_nominal(ce_mppi_planner* planner, const float* U, void* stream);
ce_status ce_mppi_get_nominal(const ce_mppi_planner* planner, float* U, void* stream);
/* Empty the obstacle history. */
ce_status ce_mppi_reset_history(ce_mppi_planner* planner, void* stream);
/* Replace the obstacle history (the {o_{t-h}} of Eq. (17)): hist is device
 * memory [h_count][n_obs][p] of obstacle centres, newest first; the planner
 * keeps the newest min(h_count, history_len) entries, exactly as if they had
 * been pushed by that many replans with n_obs obstacles (h_count = 0 empties
 * it).  The next replan pushes its own observation on top, and a different
 * obstacle count there restarts the history as usual.  Synchronises the
 * stream.  Errors: CE_EINVAL (h_count < 0, n_obs outside 0..max_obstacles,
 * NULL hist with entries), CE_EDEVICE. */
ce_status ce_mppi_set_history(ce_mppi_planner* planner, const float* hist, int32_t h_count,
                              int32_t n_obs, void* stream);
/* Set the step counter (the Philox step word of the next replan). */
ce_status ce_mppi_set_step(ce_mppi_planner* planner, uint64_t step, void* stream);
/* Checkpoint: size in bytes of the serialised state (U, history, counters). */
ce_status ce_mppi_state_size(const ce_mppi_planner* planner, size_t* bytes);
/* Serialise the state into host memory `buf` of state_size bytes; synchronises
 * the stream. */
ce_status ce_mppi_get_state(const ce_mppi_planner* planner, void* buf, size_t bytes, void* stream);
/* Restore a state produced by ce_mppi_get_state of a planner with the same
 * configuration; synchronises the stream. */
ce_status ce_mppi_set_state(ce_mppi_planner* planner, const void* buf, size_t bytes, void* stream);

/* ---- diagnostics: internal buffers of the last replan ---- */
enum {
  CE_DBG_COST = 0,       /* float [K]            S of Eq. (5)                      */
  CE_DBG_COLLIDE = 1,    /* int32 [K]            collision indicator               */
  CE_DBG_FIRST_OBS = 2,  /* int32 [K]            lowest obstacle at first contact  */
  CE_DBG_P_TERM = 3,     /* float [K][p]         p(x_{t+N})                        */
  CE_DBG_P_FIRST = 4,    /* float [K][p]         p at first contact                */
  CE_DBG_EPS = 5,        /* float [K][N][m]      applied perturbation              */
  CE_DBG_V_IDX = 6,      /* int32 [|V|]          feasible rollouts, ascending      */
  CE_DBG_Z = 7,          /* float [|V|][p]       feature of Eq. (13)               */
  CE_DBG_G = 8,          /* float [|V|][p]       direction of Eq. (15)             */
  CE_DBG_NCOUNT = 9,     /* int32 [|V|]  eps-neighbour count; exact below minPts, */
                         /*              between minPts and the count above it */
  CE_DBG_LABEL = 10,     /* int32 [|V|]          cluster label, -1 noise           */
  CE_DBG_CLUSTER_COST = 11, /* float [M]         mean cost per cluster             */
  CE_DBG_CLUSTER_DIR = 12,  /* float [M][p]      normalised mean direction Eq.(16) */
  CE_DBG_CLUSTER_SIZE = 13, /* int32 [M]                                           */
  CE_DBG_TREES = 14,        /* int32 [2]  hook-forest trees (angular runs of core  */
                            /*            buckets on the window path), 1 if the     */
                            /*            exact union-find fallback ran (> 64 trees) */
  CE_DBG_COUNT_ = 15
};
/* Copy the named buffer into device memory dst of `bytes` bytes (at most the
 * buffer's full capacity is copied; rows beyond |V| or M are unspecified). */
ce_status ce_mppi_debug_get(const ce_mppi_planner* planner, int32_t which, void* dst, size_t bytes,
                            void* stream);

/* ---- stage entry points (the same kernels on caller-supplied inputs) ---- */

/* Philox noise of the planner's configuration for rollouts 0..K-1 at `step`:
 * words  device uint32 [K][B][4], B = ceil(N*m/4) (may be NULL)
 * gauss  device float  [K][N][m] standard normals (may be NULL). */
ce_status ce_mppi_stage_noise(ce_mppi_planner* planner, uint32_t step, uint32_t* words, float* gauss,
                              void* stream);

/* Everything after the rollouts (Alg. 1 from [Pruning] on) applied to
 * rollout records supplied by the caller instead of the planner's rollout
 * kernel; the planner state (U, history, step) is used and advanced exactly
 * as by ce_mppi_replan.
 *   S [K], collide int32 [K], first_obs int32 [K], p_term [K][p],
 *   p_first [K][p], eps [K][N][m]: device. */
ce_status ce_mppi_replan_from_rollouts(ce_mppi_planner* planner, const float* x_t,
                                       const float* obstacles, int32_t n_obs, const float* S,
                                       const int32_t* collide, const int32_t* first_obs,
                                       const float* p_term, const float* p_first, const float* eps,
                                       float* u_out, float* U_out, ce_mppi_info* info,
                                       void* stream);

/* DBSCAN of the planner's kernels on V caller-supplied features z (device,
 * [V][p]) with the planner's eps/minPts; V <= K.  Outputs (device, [V]):
 * ncount (may be NULL), label; n_clusters (device int32, may be NULL). */
ce_status ce_mppi_stage_dbscan(ce_mppi_planner* planner, const float* z, int32_t V, int32_t* ncount,
                               int32_t* label, int32_t* n_clusters, void* stream);

/* ---- DBSCAN path (Sec. II-B.2) ----
 *
 * Every path computes the same clustering: closed eps-ball, minPts counting
 * the point itself, a border point in the cluster of its lowest-index core
 * neighbour, clusters numbered by their lowest core index.  The neighbour
 * relation is the same FP32 distance test on every path, so counts, labels,
 * cluster statistics and the replan's outputs are identical bit for bit;
 * only the work differs.
 *   CE_DBSCAN_WINDOW  2-D features bucketed by angle around the unit ring on
 *                     which the features of Eq. (13) lie: ring points inside
 *                     a point's inner angular window are neighbours and those
 *                     outside its outer window are not, so only the buckets
 *                     between the windows, and features off the ring, are
 *                     tested pair by pair.  About O(V) window lookups plus
 *                     the boundary tests, where the others take V^2/2 pairs.
 *                     Needs p = 2 and eps in roughly [0.01, 1.4].
 *   CE_DBSCAN_BITMAP  one tiled pass over the V^2/2 pairs into an
 *                     eps-adjacency bitmap that the later passes read;
 *                     K <= 16384.
 *   CE_DBSCAN_TILED   tiled distance passes (any K, p = 2 or 3).
 *   CE_DBSCAN_AUTO    (default) the first of these that the planner supports.
 * The mode applies to replans and to ce_mppi_stage_dbscan; a change rebuilds
 * the replan graph at the next replan.  A batch runs each 2-D member on the
 * angular windows if that is the member's path when the batch is made, and
 * every other member on the batch's spatially sorted distance passes.
 * Errors: CE_EINVAL (NULL planner, unknown mode), CE_EUNSUPPORTED (the path
 * is not available for this planner; the mode is unchanged). */
enum { CE_DBSCAN_AUTO = 0, CE_DBSCAN_WINDOW = 1, CE_DBSCAN_BITMAP = 2, CE_DBSCAN_TILED = 3 };
ce_status ce_mppi_set_dbscan_mode(ce_mppi_planner* planner, int32_t mode);
/* The path replans and stage calls use now (CE_DBSCAN_WINDOW, _BITMAP or
 * _TILED) into *path.  Errors: CE_EINVAL for NULL arguments. */
ce_status ce_mppi_get_dbscan_path(const ce_mppi_planner* planner, int32_t* path);

/* ---- allocation-free DBSCAN ----
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  It runs the
 * kernels of ce_mppi_stage_dbscan (same conventions, same results bit for bit)
 * without a planner: their per-point work arrays live in one file-scope
 * device array of the library (about 530 KB per GPU, held until the process
 * ends), so the call allocates nothing and calls no hipMalloc, hipFree or
 * allocating library routine.  The first call on a device looks up that
 * device's copy of the array (hipGetSymbolAddress).
 *
 *   device     HIP device ordinal; stream must belong to it
 *   z          device, [V][p] features (float), p = 2 or 3
 *   V          0..CE_MPPI_NOALLOC_MAX_POINTS; larger V is rejected (CE_EINVAL)
 *   eps        neighbourhood radius (closed ball), finite and > 0
 *   min_pts    minimum neighbourhood size, the point itself included, >= 1
 *   ncount     device, [V] neighbour counts (exact below min_pts, between
 *              min_pts and the exact count for core points), or NULL
 *   label      device, [V] cluster label 0..M-1 (numbered by the lowest core
 *              index), -1 noise
 *   n_clusters device, one int32 (M), or NULL
 * Asynchronous on stream.  Every call on a GPU shares that GPU's array and
 * overwrites what the previous call left there: calls that overlap on one GPU
 * (other streams or threads) race, so the caller must order them.  Errors:
 * CE_EINVAL (sizes, parameters, NULL pointers, device ordinal), CE_EDEVICE. */
#define CE_MPPI_NOALLOC_MAX_POINTS 16384
ce_status ce_mppi_dbscan_noalloc(int32_t device, const float* z, int32_t V, int32_t p, float eps,
                                 int32_t min_pts, int32_t* ncount, int32_t* label,
                                 int32_t* n_clusters, void* stream);

/* ---- launch mode and timing ---- */
enum { CE_LAUNCH_GRAPH = 0, CE_LAUNCH_DIRECT = 1 };
/* CE_LAUNCH_GRAPH (default): the first replan records the planner's kernel
 * chain into a hipGraph and every replan replays it (the first and last
 * kernels are re-pointed when the caller's buffers change).
 * CE_LAUNCH_DIRECT: every kernel of the replan is launched on the caller's
 * stream.  Both run the same kernels with the same arguments and give the
 * same bits.  Which is faster depends on the host: a replay costs the device
 * a few microseconds more than the same direct launches, while direct launches
 * cost the host a few microseconds each (see ce_mppi_tune_launch). */
ce_status ce_mppi_set_launch_mode(ce_mppi_planner* planner, int32_t mode);
/* For callers that replan back to back: run `reps` replans on (x_t,
 * obstacles) in each launch mode, timing host wall clock from the first call
 * to the stream being idle (so the slower of host submission and device work
 * counts), and keep the faster mode.  The per-call times in microseconds go
 * to *us_graph and *us_direct (either may be NULL).  u_out is a device buffer
 * of m floats that receives scratch outputs.  The persistent state (nominal,
 * history, step) is saved before and restored after each mode's run; the
 * per-rollout diagnostic buffers hold the last replan's values.
 * Synchronises the stream.  Errors: CE_EINVAL for NULL pointers, reps outside
 * [1, 10000] or bad n_obs; CE_EDEVICE for HIP failures. */
ce_status ce_mppi_tune_launch(ce_mppi_planner* planner, const float* x_t, const float* obstacles,
                              int32_t n_obs, float* u_out, int32_t reps, void* stream,
                              double* us_graph, double* us_direct);
/* capacity > 0: the next `capacity` replans are launched directly with HIP
 * events recorded on the replan stream before the rollout kernel, after it
 * and after the last kernel; 0 disables.  Allocates the events. */
ce_status ce_mppi_timing_enable(ce_mppi_planner* planner, int32_t capacity);
/* Sums (ms) over the timed replans of the rollout kernel, of everything after
 * it and of the whole replan, and their count; waits for the events. */
ce_status ce_mppi_timing_read(ce_mppi_planner* planner, double* rollout_ms, double* post_ms,
                              double* total_ms, int32_t* count);

/* The same per timed replan, in order: host arrays of cap entries receive
 * the rollout, post-rollout and total times (ms) of the first
 * min(cap, count) timed replans; *count (may be NULL) receives the number of
 * timed replans.  Waits for the events.  Errors: CE_EINVAL for NULL arrays
 * with cap > 0 or cap < 0; CE_EDEVICE. */
ce_status ce_mppi_timing_read_each(ce_mppi_planner* planner, int32_t cap, double* rollout_ms,
                                   double* post_ms, double* total_ms, int32_t* count);

/* Time the rollout phase alone: `reps` back-to-back launches of the rollout
 * kernel of a replan on (x_t, obstacles) between two HIP events on `stream`;
 * *ms_per_launch receives the mean time per launch.  Device pointers as in
 * ce_mppi_replan.  The planner's persistent state (nominal sequence,
 * observation history, step counter) is saved before and restored after, so
 * the next replan is unaffected; the per-rollout diagnostic buffers hold the
 * last launch's values.  Synchronises the stream.  Errors: CE_EINVAL for
 * NULL pointers or reps outside [1, 100000]; CE_EDEVICE for HIP failures. */
ce_status ce_mppi_time_rollout(ce_mppi_planner* planner, const float* x_t, const float* obstacles,
                               int32_t n_obs, int32_t reps, void* stream, double* ms_per_launch);

/* ---- batched form: many planners per launch ----
 *
 * A batch runs one replan of each of its planners (Alg. 1 for every member,
 * each exactly as ce_mppi_replan would run it) as one graph launch.  Every
 * phase of the replan is one persistent kernel per planner kind (rollout
 * kind: unicycle on 32 or 64 lanes, arm; DBSCAN kind: 2-D on the angular
 * windows, 2-D on sorted distance passes, 3-D) whose fixed grid loops over
 * the work items of all members; the DBSCAN work tables are sized on the
 * device from each member's feasible count.  The results of a member are
 * bitwise those of ce_mppi_replan on the same inputs and state.
 *
 * Ownership: the batch holds references to its planners, which must outlive
 * it, stay on the batch's device, and must not run a replan concurrently with
 * a batch replan.  The batch owns a small device table (about 1 KB per
 * member) and a pinned staging buffer for the per-call pointers. */
typedef struct ce_mppi_batch ce_mppi_batch;

/* Per-member inputs and outputs of one batch replan; the pointers are device
 * pointers with the layouts of ce_mppi_replan. */
typedef struct ce_mppi_batch_io {
  const float* x_t;        /* [n] current state                                */
  const float* obstacles;  /* [n_obs][p+1] (centre, radius), or NULL if n_obs=0 */
  int32_t n_obs;           /* 0 .. the member's max_obstacles                   */
  int32_t reserved;        /* must be 0                                         */
  float* u_out;            /* [m] applied control (required)                    */
  float* U_out;            /* [N][m] updated sequence before the shift, or NULL */
  void* info;              /* ce_mppi_info, or NULL                             */
} ce_mppi_batch_io;

/* Launch shapes of a batch (chosen by ce_mppi_batch_autotune or set). */
typedef struct ce_mppi_batch_tuning {
  int32_t colg;               /* column tiles per DBSCAN count item: 1,2,4 or 8 */
  int32_t tile_blocks_per_cu; /* persistent blocks per CU, tiled DBSCAN: 1..16  */
  int32_t roll_blocks_per_cu; /* persistent blocks per CU, rollouts: 1..8       */
  int32_t roll_per_wave;      /* rollouts per wave per work item: 1, 2, 4 or 8  */
} ce_mppi_batch_tuning;

/* Create a batch of n distinct planners (1 <= n <= CE_MPPI_MAX_BATCH) on the
 * same device, with the default tuning (colg 8, 8 tile blocks and 4 rollout
 * blocks per CU, 4 rollouts per wave).  Errors: CE_EINVAL (NULL, duplicates, mixed devices, n out
 * of range), CE_ENOMEM, CE_EDEVICE. */
ce_status ce_mppi_batch_create(ce_mppi_planner* const* planners, int32_t n, ce_mppi_batch** out);
void ce_mppi_batch_destroy(ce_mppi_batch* batch);

/* One replan of every member on `stream` (asynchronous).  io: host array of
 * n entries, read during the call; the per-call pointers are uploaded only
 * when they differ from the previous call's.  Errors: CE_EINVAL for a NULL
 * u_out or x_t, n_obs out of range, or a nonzero reserved field;
 * CE_EDEVICE for HIP failures. */
ce_status ce_mppi_batch_replan(ce_mppi_batch* batch, const ce_mppi_batch_io* io, void* stream);

/* One replan of the listed members only (continuous batching): members[q]
 * indexes the planner list given at creation (distinct), io[q] is its
 * inputs/outputs.  The work tables of the subset are built on the host and
 * uploaded with the pointers; launches rotate over three table areas, and a
 * call waits (host side) until the area it reuses has finished its previous
 * launch, so up to three subset launches can be in flight on different
 * streams.  Members of launches in flight must not be listed again until
 * those launches have finished (each member's replans are sequential).
 * Errors: CE_EINVAL for NULL, out-of-range or repeated members and the io
 * errors of ce_mppi_batch_replan; CE_EDEVICE for HIP failures. */
ce_status ce_mppi_batch_replan_subset(ce_mppi_batch* batch, const int32_t* members, int32_t count,
                                      const ce_mppi_batch_io* io, void* stream);

ce_status ce_mppi_batch_set_tuning(ce_mppi_batch* batch, const ce_mppi_batch_tuning* tuning);
ce_status ce_mppi_batch_get_tuning(const ce_mppi_batch* batch, ce_mppi_batch_tuning* tuning);

/* Project-written autotuner: times `reps` batch replans on io per candidate
 * shape, first the rollout shape (rollouts per wave in {1,2,4,8} x rollout
 * blocks per CU in {2,4}), then the DBSCAN shape (colg in {2,4,8} x tile
 * blocks per CU in {4,8,16}); keeps the fastest and returns it with its mean
 * time per batch replan.  Results do not depend on the shape: every member's
 * output is bitwise the same under every tuning.  The members' states are saved before and
 * restored after every candidate, so the batch continues from where it was.
 * Synchronises the stream. */
ce_status ce_mppi_batch_autotune(ce_mppi_batch* batch, const ce_mppi_batch_io* io, int32_t reps,
                                 void* stream, ce_mppi_batch_tuning* best, double* best_ms);

/* ---- served form: continuous batching over resident sessions ----
 *
 * A server owns planner sessions (each a planner whose nominal sequence and
 * observation history stay on the device between requests) and a scheduler
 * thread.  Replan requests carry host inputs; the scheduler launches the
 * pending requests of idle sessions together (one batched replan over those
 * members, ce_mppi_batch_replan_subset), in arrival order, at most one request
 * per session per launch and max_batch per launch, with up to max_inflight
 * launches running at once on their own streams.  Every request's result is
 * bitwise the one a plain ce_mppi_replan of its session would give for the
 * same sequence of requests.  Sessions are admitted while their device memory
 * (the planner arena) fits memory_budget; every buffer a request needs
 * (staging, outputs) is allocated at start, so requests are admitted as
 * launch slots free up, without allocating.
 *
 * A launch of one or two requests runs each through its session's own
 * single-planner replan (ce_mppi_replan, in the launch mode ce_mppi_tune_launch
 * picks for each session at start) instead of the batched chain: fewer
 * kernels, the same results.
 *
 * CE_SERVE_PLAIN is the one-request-per-launch form for comparison: the
 * scheduler serves one request at a time with ce_mppi_replan on the
 * session's planner (the single-planner kernels, in the launch mode that
 * ce_mppi_tune_launch picks for each session at start); max_batch and
 * max_inflight must be 1. */
typedef struct ce_mppi_server ce_mppi_server;

enum { CE_SERVE_BATCHED = 0, CE_SERVE_PLAIN = 1 };

typedef struct ce_mppi_server_config {
  int32_t device;
  int32_t max_batch;       /* requests per launch, 1..CE_MPPI_MAX_BATCH (1: one per launch) */
  int32_t max_inflight;    /* launches in flight, 1..3                                      */
  int32_t mode;            /* CE_SERVE_BATCHED (0) or CE_SERVE_PLAIN                        */
  uint64_t memory_budget;  /* device bytes the sessions may hold; 0: 90 % of free memory    */
} ce_mppi_server_config;

typedef struct ce_mppi_server_stats {
  uint64_t launches, served;
  double mean_batch;        /* requests per launch */
  int32_t max_batch, max_inflight, sessions, reserved;
  uint64_t session_bytes, budget_bytes;
} ce_mppi_server_stats;

ce_status ce_mppi_server_create(const ce_mppi_server_config* cfg, ce_mppi_server** out);

/* Open a session (before start) with the planner configuration cfg on the
 * server's device and, if U0 is not NULL, the host nominal sequence [N][m].
 * Returns its id (0, 1, ...).  CE_EBUSY when its memory would exceed the
 * budget (or 1024 sessions are open); CE_EINVAL after start. */
ce_status ce_mppi_server_open_session(ce_mppi_server* server, const ce_mppi_config* cfg,
                                      const float* U0, int32_t* session);

/* Freeze the session set and start the scheduler thread. */
ce_status ce_mppi_server_start(ce_mppi_server* server);

/* Queue one replan of `session` with host inputs x_t [n] and obstacles
 * [n_obs][p+1] (copied before return); *ticket identifies the request.
 * Thread-safe. */
ce_status ce_mppi_server_submit(ce_mppi_server* server, int32_t session, const float* x_t,
                                const float* obstacles, int32_t n_obs, uint64_t* ticket);

/* Block until the request is served: u_out [m] and info (host, may be NULL)
 * receive its outputs, latency_s (may be NULL) the time from submission to
 * completion.  A ticket is waited for once.  Thread-safe. */
ce_status ce_mppi_server_wait(ce_mppi_server* server, uint64_t ticket, float* u_out,
                              ce_mppi_info* info, double* latency_s);

/* Load generator: submit request i at t_arrival[i] seconds after the call
 * (ascending), for session[i], with state x_t[i*12 .. ] and obstacles rows
 * packed from obstacles[i*256 .. ] (n_obs[i] rows of p+1 floats; NULL if no
 * request has obstacles), then wait for all; latency_s[i] and u_out[i*6 ..]
 * (host, may be NULL) receive the results. */
ce_status ce_mppi_server_run_trace(ce_mppi_server* server, int32_t n, const double* t_arrival,
                                   const int32_t* session, const float* x_t, const float* obstacles,
                                   const int32_t* n_obs, double* latency_s, float* u_out);

ce_status ce_mppi_server_get_stats(ce_mppi_server* server, ce_mppi_server_stats* out);

/* The planner of a session (owned by the server), e.g. for its diagnostics or
 * state; NULL for an unknown session.  Not to be replanned while the server
 * runs. */
ce_mppi_planner* ce_mppi_server_session_planner(ce_mppi_server* server, int32_t session);

/* Stop the scheduler after serving the pending requests, free everything. */
void ce_mppi_server_destroy(ce_mppi_server* server);

/* ---- errors ---- */
const char* ce_mppi_status_string(ce_status status);
/* Message of the last failed call on this thread ("" if none). */
const char* ce_mppi_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CEMPPI_H */
