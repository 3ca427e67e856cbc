/*
 * cemppi_oracle.h -- plain FP64 CPU reference for one CE-MPPI replan.
 *
 * TEST INFRASTRUCTURE.  This library exists only so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU path
 * against an obviously-correct implementation written from the paper
 * (Liu, Chang, Chen: "Clustering-Embedded Model Predictive Path Integral
 * Control", Sec. II and Alg. 1).  The product path never links, loads or
 * calls it, and it shares no code, header, table or helper with the GPU
 * library.
 *
 * Precision.  Every value and every decision is computed in double
 * precision from the single-precision parameters promoted exactly: the
 * collision flag (squared distance against the squared sum of radii), the
 * DBSCAN neighbourhood (squared distance against eps squared), the closest
 * obstacle, the dynamic-rule threshold and the two cluster argmins.  A
 * single-precision implementation can decide differently only where the
 * compared quantities lie within its rounding of each other; the oracle
 * reports the quantities that let a caller find those cases (boundary
 * clearance per rollout, the closest-obstacle margin, the selection margin).
 *
 * Layouts are row-major and dense.  All arrays are owned by the caller.
 */
#ifndef CEMPPI_ORACLE_H
#define CEMPPI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_M 6
#define ORC_MAX_OBS 64

/* Dynamics instances f(.) of Sec. II-A: the differential-drive robot of
 * Sec. III-A (n=3, m=2, p=2) and a six-joint serial arm driven by joint
 * velocities as in Sec. III-C (n=12, m=6, p=3). */
enum { ORC_UNICYCLE = 0, ORC_ARM6 = 1 };
enum { ORC_STATIC = 0, ORC_DYNAMIC = 1 };
enum { ORC_REF_TERMINAL = 0, ORC_REF_FIRST_CONTACT = 1 };

/* Optional variants (orc_problem.flags).
 * ORC_FLAG_POSE_COST (arm only): the goal-reaching stage cost of the
 *   real-robot experiment, Sec. III-C: w_p |p_ee - p_g| + w_R d_R(R_ee, R_g)
 *   + w_c I_col(q_t), with (w_p, w_R, w_c) = (Q[0], Q[1], Q[2]) on the stage
 *   states x_0..x_{N-1} and (Qf[0], Qf[1], Qf[2]) on x_N.  R_g is given as a
 *   rotation vector (axis times angle, radians) in goal[3..5]; d_R is the
 *   angle of the relative rotation, from unit quaternions.  The control and
 *   joint-limit terms stay as in the default cost.
 * ORC_FLAG_OBS_CONST_VEL: inside the rollouts every obstacle moves with its
 *   own constant velocity, estimated as in Eq. (17) from the observation
 *   history; state x_j is tested against the obstacles at time j dt.  The
 *   default keeps the obstacles where they were observed. */
#define ORC_FLAG_POSE_COST 1u
#define ORC_FLAG_OBS_CONST_VEL 2u

/* branch taken by Alg. 1 */
enum { ORC_BRANCH_CLUSTER = 0, ORC_BRANCH_FALLBACK = 1, ORC_BRANCH_ALL_COLLIDE = 2 };

/* status bits */
#define ORC_ST_FALLBACK 1u        /* no colliding rollout: plain MPPI (Alg. 1 fallback) */
#define ORC_ST_ALL_COLLIDE 2u     /* every rollout collides: plain MPPI over all K      */
#define ORC_ST_NO_CLUSTER 4u      /* DBSCAN found no cluster: update over all of V      */
#define ORC_ST_DYN_STATIC 8u      /* dynamic rule impossible (H'<2 or slow obstacle)    */
#define ORC_ST_NONFINITE 16u      /* non-finite input: replan is a no-op                */

typedef struct orc_problem {
  int32_t dynamics;         /* ORC_UNICYCLE or ORC_ARM6                          */
  int32_t N;                /* horizon                                            */
  int32_t K;                /* number of rollouts                                 */
  double dt;                /* integration step (also the observation interval)  */
  double lambda;            /* temperature, > 0                                   */
  double L[36];             /* noise Cholesky factor, m x m row-major, Sigma=LL^T */
  double u_min[6], u_max[6];/* control bounds; +-INFINITY disables the clamp      */
  double dbscan_eps;        /* DBSCAN radius (closed ball)                        */
  int32_t dbscan_min_pts;   /* DBSCAN minPts, the point itself included           */
  double norm_eps;          /* the small epsilon of the normalisations            */
  int32_t scene_mode;       /* ORC_STATIC / ORC_DYNAMIC                           */
  int32_t history_len;      /* H                                                  */
  double v_obs_min;         /* below this obstacle speed the static rule is used  */
  int32_t ref_mode;         /* ORC_REF_TERMINAL / ORC_REF_FIRST_CONTACT           */
  double robot_radius;      /* unicycle body radius (0: point robot)              */
  double goal[6];           /* unicycle: x_f; arm: end-effector target p_g        */
  double Q[6], R[6], Qf[6]; /* diagonal stage-state, stage-control, terminal     */
  double dh[6][4];          /* arm: per joint (a, d, alpha, theta offset)         */
  int32_t n_link_spheres;   /* arm: collision spheres along the link chain        */
  double link_sphere_radius;
  double q_limit[6];        /* arm: joint-limit penalty threshold                 */
  double w_limit;           /* arm: joint-limit penalty weight                    */
  uint64_t seed;            /* Philox key                                         */
  uint32_t stream_id;       /* Philox counter word 3                              */
  uint32_t flags;           /* ORC_FLAG_* bits                                    */
} orc_problem;

/* Outputs of orc_replan.  Every pointer may be NULL (not produced).
 * Per-rollout arrays have K rows; the compacted arrays (v_idx, z, g, ncount,
 * core, label) have n_feas valid rows; cluster arrays have n_clusters rows
 * (capacity c_cap). */
typedef struct orc_out {
  double* S;           /* [K]        trajectory cost, Eq. (5)                     */
  int32_t* col;        /* [K]        collision indicator                         */
  int32_t* first_obs;  /* [K]        lowest obstacle hit at the first hit step    */
  double* p_term;      /* [K][p]     p(x_{t+N})                                  */
  double* p_first;     /* [K][p]     p at the first colliding state              */
  double* eps_eff;     /* [K][N][m]  applied perturbation (clamped - nominal)    */
  double* clearance;   /* [K]        min over states/obstacles of |dist-R|/R     */
  int32_t* v_idx;      /* [K]        feasible rollout indices, ascending         */
  double* z;           /* [K][p]     clustering feature of each feasible rollout */
  double* g;           /* [K][p]     unit terminal displacement, Eq. (15)        */
  int32_t* ncount;     /* [K]        eps-neighbour count (self included)         */
  int32_t* core;       /* [K]        core flag                                   */
  int32_t* label;      /* [K]        cluster label 0..M-1, -1 noise              */
  int32_t c_cap;       /* capacity of the cluster arrays                          */
  double* c_mean_cost; /* [c_cap]    mean cost per cluster                        */
  double* c_dir;       /* [c_cap][p] normalised mean direction, Eq. (16)          */
  int32_t* c_size;     /* [c_cap]                                                 */
  int32_t closest_force; /* in: -2 computes o*; -1 or an obstacle index is taken as o*
                            (resolves a near tie the way another implementation did)  */
  double* weight;      /* [K]        normalised update weight of each rollout     */
  double* U_new;       /* [N][m]     updated nominal sequence                     */
  double* U_next;      /* [N][m]     shifted warm start for the next replan       */
  double* u_out;       /* [m]        control to apply                             */
  /* scalars (always written) */
  int32_t branch, n_col, n_feas, n_ref, n_clusters, selected, selected_size;
  int32_t closest, rule, h_used;
  uint32_t status;
  double margin;
  double closest_margin; /* second-smallest minus smallest surface clearance at x_t */
  double ref_point[3];
  double v_obs[3];
  double v_obs_hat[3];
  double s_min;
} orc_out;

/* ---- primitives (exported for the tests that pin them) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t w);
void orc_box_muller(uint32_t wa, uint32_t wb, double* ga, double* gb);
int32_t orc_noise_blocks(int32_t N, int32_t m);
void orc_noise_words(const orc_problem* P, uint32_t step, int32_t k, uint32_t* words);
void orc_rollout_noise(const orc_problem* P, uint32_t step, int32_t k, double* gauss, double* eps);
int32_t orc_dims(int32_t dynamics, int32_t* n, int32_t* m, int32_t* p);

void orc_unicycle_step(const double x[3], const double u[2], double dt, double xn[3]);
void orc_arm_frames(const double q[6], const double dh[6][4], double origins[7][3], double rot[3][3]);
void orc_arm_spheres(const double origins[7][3], int32_t ns, double* centres);

/* Orientation error of the arm's pose cost (Sec. III-C): unit quaternions
 * (w, x, y, z) of a rotation vector and of a rotation matrix, and the angle
 * 2 acos |<a, b>| between two orientations, in [0, pi]. */
void orc_rotvec_quat(const double r[3], double q[4]);
void orc_rot_quat(const double R[3][3], double q[4]);
double orc_quat_angle(const double a[4], const double b[4]);

/* One rollout from x0 with applied controls ut[N][m]: fills traj[(N+1)][n]
 * (may be NULL), returns cost, collision flag, first-hit obstacle, terminal
 * and first-contact points and the boundary clearance. */
void orc_simulate(const orc_problem* P, const double* x0, const double* ut, const double* obs,
                  int32_t n_obs, double* traj, double* S, int32_t* col, int32_t* first_obs,
                  double* p_term, double* p_first, double* clearance);

/* orc_simulate with moving obstacles: obstacle i is at obs_i + j dt vel_i
 * when state x_j is tested (vel [n_obs][p]; NULL = frozen). */
void orc_simulate_moving(const orc_problem* P, const double* x0, const double* ut,
                         const double* obs, const double* vel, int32_t n_obs, double* traj,
                         double* S, int32_t* col, int32_t* first_obs, double* p_term,
                         double* p_first, double* clearance);

int32_t orc_closest_obstacle(const orc_problem* P, const double* x0, const double* obs, int32_t n_obs);
int32_t orc_closest_obstacle_margin(const orc_problem* P, const double* x0, const double* obs,
                                    int32_t n_obs, double* margin);
void orc_obstacle_velocity(const double* hist, int32_t h_avail, int32_t n_obs, int32_t p, int32_t idx,
                           int32_t H, double dt, double v[3]);

int32_t orc_dbscan(const double* z, int32_t V, int32_t p, double eps, int32_t min_pts,
                   int32_t* ncount, int32_t* core, int32_t* label);

/* Cluster statistics and selection (Alg. 1 [Cluster stats], [Selection],
 * Eq. (14)-(18)) on given labels of the nV feasible rollouts (M >= 1
 * clusters), their costs S_v [nV] and directions g [nV][p]; closest is o*.
 * Writes the cluster arrays and the selection fields of *out (c_cap and the
 * array pointers must be set); returns the selected label. */
int32_t orc_select_cluster(const orc_problem* P, int32_t nV, const int32_t* label, int32_t M,
                           const double* S_v, const double* g, const double* hist, int32_t h_avail,
                           int32_t n_obs, int32_t closest, orc_out* out);

void orc_weighted_update(int32_t n_set, const int32_t* set, const double* S, const double* eps_eff,
                         int32_t N, int32_t m, double lambda, const double* U, double* U_new,
                         double* weight_out, double* s_min);

/* Full replan, Alg. 1.  hist holds h_avail observations of the obstacle
 * positions, newest first ([h_avail][n_obs][p]); hist[0] must equal the
 * positions in obs.  Returns 0, or -1 on invalid arguments. */
int32_t orc_replan(const orc_problem* P, const double* x_t, const double* U, const double* obs,
                   int32_t n_obs, const double* hist, int32_t h_avail, uint32_t step, orc_out* out);

/* Alg. 1 from [Pruning] on, applied to given rollout records (S [K],
 * col [K], first_obs [K], p_term [K][p], p_first [K][p], eps_eff [K][N][m]);
 * per-rollout outputs of `out` are not written. */
int32_t orc_replan_from_rollouts(const orc_problem* P, const double* x_t, const double* U,
                                 const double* obs, int32_t n_obs, const double* hist,
                                 int32_t h_avail, const double* S, const int32_t* col,
                                 const int32_t* first_obs, const double* p_term,
                                 const double* p_first, const double* eps_eff, orc_out* out);

#ifdef __cplusplus
}
#endif
#endif
