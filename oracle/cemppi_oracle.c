/*
 * cemppi_oracle.c -- plain FP64 CPU reference for one CE-MPPI replan.
 *
 * TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use this file.  It is written from the paper (Sec. II,
 * Alg. 1, Sec. III) as slow scalar loops, in the paper's order, so that it
 * can be read against the equations.  No blocking, fusion or reordering.
 *
 * Readings where the paper is silent:
 *  - noise: Philox4x32-10 counter layout (block, rollout, step, stream) and
 *    Box-Muller on 24-bit uniforms; Sigma given as its Cholesky factor L;
 *  - controls are clamped to the bounds and the applied perturbation
 *    (clamped control minus nominal) enters the update;
 *  - collisions are checked on the states j = 1..N against obstacles frozen
 *    at their current positions, or, with the constant-velocity flag, moved
 *    by j dt times each obstacle's own Eq. (17) velocity;
 *  - the pose cost (flag) uses the geodesic angle between the end-effector
 *    and goal orientations, and its contact term shares the collision test;
 *  - the reference point averages the colliding rollouts whose first hit is
 *    the obstacle closest to x_t, and all colliding rollouts if none is;
 *  - DBSCAN: closed eps-ball, minPts counts the point itself, a border
 *    point joins the cluster of its lowest-index core neighbour, clusters are
 *    numbered by their lowest core index;
 *  - no cluster -> update over every feasible rollout; no feasible rollout
 *    -> plain MPPI over all K;
 *  - the shift repeats the last control.
 */
#include "cemppi_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10, as defined by Salmon, Moraes, Dror and Shaw,          */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of */
/* two 32x32->64 multiplications with the round keys bumped by the Weyl */
/* constants between rounds.                                            */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* Uniform in the open interval (0,1) from the top 23 bits of a word:
 * (2*(w>>9)+1) * 2^-24.  Exactly representable in single precision. */
double orc_uniform(uint32_t w) { return (2.0 * (double)(w >> 9) + 1.0) * (1.0 / 16777216.0); }

/* Box-Muller transform (Box & Muller, 1958). */
void orc_box_muller(uint32_t wa, uint32_t wb, double* ga, double* gb) {
  const double PI = 3.14159265358979323846;
  double ua = orc_uniform(wa), ub = orc_uniform(wb);
  double r = sqrt(-2.0 * log(ua));
  *ga = r * cos(2.0 * PI * ub);
  *gb = r * sin(2.0 * PI * ub);
}

int32_t orc_dims(int32_t dynamics, int32_t* n, int32_t* m, int32_t* p) {
  if (dynamics == ORC_UNICYCLE) {
    *n = 3; *m = 2; *p = 2;
    return 0;
  }
  if (dynamics == ORC_ARM6) {
    *n = 12; *m = 6; *p = 3;
    return 0;
  }
  return -1;
}

int32_t orc_noise_blocks(int32_t N, int32_t m) { return (N * m + 3) / 4; }

/* Philox words of rollout k: block b has counter (b, k, step, stream_id)
 * and key (seed low word, seed high word). */
void orc_noise_words(const orc_problem* P, uint32_t step, int32_t k, uint32_t* words) {
  int32_t n, m, p;
  orc_dims(P->dynamics, &n, &m, &p);
  int32_t B = orc_noise_blocks(P->N, m);
  uint32_t key[2] = {(uint32_t)(P->seed & 0xffffffffu), (uint32_t)(P->seed >> 32)};
  for (int32_t b = 0; b < B; ++b) {
    uint32_t ctr[4] = {(uint32_t)b, (uint32_t)k, step, P->stream_id};
    orc_philox4x32_10(ctr, key, words + 4 * b);
  }
}

/* Gaussian perturbations of rollout k (Sec. II-A: eps ~ N(0, Sigma)).
 * Element e = j*m + i of the flattened [N][m] sequence is standard normal
 * g_e; elements (2q, 2q+1) come from one Box-Muller pair fed by words
 * (0,1) of block q/2 when q is even and words (2,3) when q is odd.
 * eps_j = L g_j. */
void orc_rollout_noise(const orc_problem* P, uint32_t step, int32_t k, double* gauss, double* eps) {
  int32_t n, m, p;
  orc_dims(P->dynamics, &n, &m, &p);
  int32_t N = P->N, E = N * m;
  int32_t B = orc_noise_blocks(N, m);
  uint32_t* words = (uint32_t*)malloc(sizeof(uint32_t) * 4 * (size_t)B);
  double* g = (double*)malloc(sizeof(double) * (size_t)(4 * B));
  orc_noise_words(P, step, k, words);
  for (int32_t q = 0; 2 * q < E; ++q) {
    int32_t b = q / 2, h = q % 2;
    orc_box_muller(words[4 * b + 2 * h], words[4 * b + 2 * h + 1], &g[2 * q], &g[2 * q + 1]);
  }
  for (int32_t j = 0; j < N; ++j) {
    for (int32_t i = 0; i < m; ++i) {
      double s = 0.0;
      for (int32_t c = 0; c <= i; ++c) s += P->L[i * m + c] * g[j * m + c];
      if (eps) eps[j * m + i] = s;
      if (gauss) gauss[j * m + i] = g[j * m + i];
    }
  }
  free(g);
  free(words);
}

/* ------------------------------------------------------------------ */
/* Dynamics                                                           */
/* ------------------------------------------------------------------ */

/* Differential-drive kinematics, Sec. III-A, Eq. (21): explicit Euler with
 * the heading taken at the start of the step. */
void orc_unicycle_step(const double x[3], const double u[2], double dt, double xn[3]) {
  xn[0] = x[0] + u[0] * cos(x[2]) * dt;
  xn[1] = x[1] + u[0] * sin(x[2]) * dt;
  xn[2] = x[2] + u[1] * dt;
}

static void mat4_mul(const double A[4][4], const double B[4][4], double C[4][4]) {
  double T[4][4];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int i = 0; i < 4; ++i) s += A[r][i] * B[i][c];
      T[r][c] = s;
    }
  memcpy(C, T, sizeof(T));
}

static void mat4_identity(double A[4][4]) {
  memset(A, 0, sizeof(double) * 16);
  for (int i = 0; i < 4; ++i) A[i][i] = 1.0;
}

/* Standard Denavit-Hartenberg chain: joint i contributes
 * Rz(q_i + offset_i) * Tz(d_i) * Tx(a_i) * Rx(alpha_i), each as a full 4x4
 * homogeneous transform.  origins[0] is the base origin, origins[i] the
 * origin of frame i; origins[6] is the end effector p_ee(q) of Sec. III-C. */
void orc_arm_frames(const double q[6], const double dh[6][4], double origins[7][3], double rot[3][3]) {
  double T[4][4];
  mat4_identity(T);
  origins[0][0] = origins[0][1] = origins[0][2] = 0.0;
  for (int i = 0; i < 6; ++i) {
    double a = dh[i][0], d = dh[i][1], alpha = dh[i][2], th = q[i] + dh[i][3];
    double Rz[4][4], Tz[4][4], Tx[4][4], Rx[4][4];
    mat4_identity(Rz);
    Rz[0][0] = cos(th); Rz[0][1] = -sin(th);
    Rz[1][0] = sin(th); Rz[1][1] = cos(th);
    mat4_identity(Tz);
    Tz[2][3] = d;
    mat4_identity(Tx);
    Tx[0][3] = a;
    mat4_identity(Rx);
    Rx[1][1] = cos(alpha); Rx[1][2] = -sin(alpha);
    Rx[2][1] = sin(alpha); Rx[2][2] = cos(alpha);
    mat4_mul(T, Rz, T);
    mat4_mul(T, Tz, T);
    mat4_mul(T, Tx, T);
    mat4_mul(T, Rx, T);
    origins[i + 1][0] = T[0][3];
    origins[i + 1][1] = T[1][3];
    origins[i + 1][2] = T[2][3];
  }
  if (rot)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) rot[r][c] = T[r][c];
}

/* Collision spheres of the arm: ns centres spread along the polyline of
 * frame origins P0..P6 at arc-length fractions (s + 1/2) / ns. */
void orc_arm_spheres(const double origins[7][3], int32_t ns, double* centres) {
  double seg[6], total = 0.0;
  for (int i = 0; i < 6; ++i) {
    double dx = origins[i + 1][0] - origins[i][0];
    double dy = origins[i + 1][1] - origins[i][1];
    double dz = origins[i + 1][2] - origins[i][2];
    seg[i] = sqrt(dx * dx + dy * dy + dz * dz);
    total += seg[i];
  }
  for (int32_t s = 0; s < ns; ++s) {
    double target = ((double)s + 0.5) / (double)ns * total;
    int i = 0;
    double start = 0.0;
    while (i < 5 && start + seg[i] < target) {
      start += seg[i];
      ++i;
    }
    double t = seg[i] > 0.0 ? (target - start) / seg[i] : 0.0;
    for (int c = 0; c < 3; ++c)
      centres[3 * s + c] = origins[i][c] + t * (origins[i + 1][c] - origins[i][c]);
  }
}

/* ------------------------------------------------------------------ */
/* Orientation error of the arm's pose cost (Sec. III-C)              */
/* ------------------------------------------------------------------ */

/* Unit quaternion (w, x, y, z) of the rotation by angle |r| about r/|r|:
 * (cos(|r|/2), sin(|r|/2) r/|r|); the identity for r = 0. */
void orc_rotvec_quat(const double r[3], double q[4]) {
  double th = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (th == 0.0) {
    q[0] = 1.0;
    q[1] = q[2] = q[3] = 0.0;
    return;
  }
  double s = sin(0.5 * th) / th;
  q[0] = cos(0.5 * th);
  q[1] = s * r[0];
  q[2] = s * r[1];
  q[3] = s * r[2];
}

/* Unit quaternion of a rotation matrix.  The four quantities
 * 4w^2 = 1 + R00 + R11 + R22, 4x^2 = 1 + R00 - R11 - R22, and so on, are
 * compared and the largest component is recovered from its square root; the
 * others follow from the off-diagonal sums and differences, divided by it.
 * The sign of q is arbitrary (q and -q are the same rotation). */
void orc_rot_quat(const double R[3][3], double q[4]) {
  double d[4] = {1.0 + R[0][0] + R[1][1] + R[2][2], 1.0 + R[0][0] - R[1][1] - R[2][2],
                 1.0 - R[0][0] + R[1][1] - R[2][2], 1.0 - R[0][0] - R[1][1] + R[2][2]};
  int b = 0;
  for (int i = 1; i < 4; ++i)
    if (d[i] > d[b]) b = i;
  double f = 0.5 * sqrt(d[b]); /* the largest |component| */
  double k = 0.25 / f;
  switch (b) {
    case 0:
      q[0] = f;
      q[1] = (R[2][1] - R[1][2]) * k;
      q[2] = (R[0][2] - R[2][0]) * k;
      q[3] = (R[1][0] - R[0][1]) * k;
      break;
    case 1:
      q[1] = f;
      q[0] = (R[2][1] - R[1][2]) * k;
      q[2] = (R[0][1] + R[1][0]) * k;
      q[3] = (R[0][2] + R[2][0]) * k;
      break;
    case 2:
      q[2] = f;
      q[0] = (R[0][2] - R[2][0]) * k;
      q[1] = (R[0][1] + R[1][0]) * k;
      q[3] = (R[1][2] + R[2][1]) * k;
      break;
    default:
      q[3] = f;
      q[0] = (R[1][0] - R[0][1]) * k;
      q[1] = (R[0][2] + R[2][0]) * k;
      q[2] = (R[1][2] + R[2][1]) * k;
      break;
  }
}

/* Angle between two orientations given as unit quaternions: the relative
 * rotation a^-1 b has scalar part <a, b>, so its angle is 2 acos |<a, b>|. */
double orc_quat_angle(const double a[4], const double b[4]) {
  double c = fabs(a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3]);
  if (c > 1.0) c = 1.0;
  return 2.0 * acos(c);
}

/* ------------------------------------------------------------------ */
/* Cost terms, Eq. (5) with the instances of Sec. III                  */
/* ------------------------------------------------------------------ */

static double limit_penalty(const orc_problem* P, const double* q) {
  double s = 0.0;
  for (int i = 0; i < 6; ++i) {
    double e = fabs(q[i]) - P->q_limit[i];
    if (e > 0.0) s += e * e;
  }
  return P->w_limit * s;
}

static double sqdist(const double* a, const double* b, int32_t p) {
  double s = 0.0;
  for (int32_t i = 0; i < p; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
  return s;
}

/* Pose terms of the real-robot cost (Sec. III-C) at joint angles q, with
 * weights w = (w_p, w_R, w_c) and the collision indicator icol. */
static double pose_terms(const orc_problem* P, const double* q, const double* w, int32_t icol) {
  double org[7][3], rot[3][3], qe[4], qg[4];
  orc_arm_frames(q, P->dh, org, rot);
  orc_rot_quat(rot, qe);
  orc_rotvec_quat(P->goal + 3, qg);
  return w[0] * sqrt(sqdist(org[6], P->goal, 3)) + w[1] * orc_quat_angle(qe, qg) +
         w[2] * (double)icol;
}

/* stage cost l(x, u); icol is I_col(x), used by the pose cost only */
static double stage_cost(const orc_problem* P, const double* x, const double* u, int32_t icol) {
  double s = 0.0;
  if (P->dynamics == ORC_UNICYCLE) {
    for (int i = 0; i < 3; ++i) s += P->Q[i] * (x[i] - P->goal[i]) * (x[i] - P->goal[i]);
    for (int i = 0; i < 2; ++i) s += P->R[i] * u[i] * u[i];
  } else {
    if (P->flags & ORC_FLAG_POSE_COST) {
      s += pose_terms(P, x, P->Q, icol);
    } else {
      double org[7][3];
      orc_arm_frames(x, P->dh, org, NULL);
      s += P->Q[0] * sqdist(org[6], P->goal, 3);
    }
    s += limit_penalty(P, x);
    for (int i = 0; i < 6; ++i) s += P->R[i] * u[i] * u[i];
  }
  return s;
}

/* terminal cost phi(x) */
static double terminal_cost(const orc_problem* P, const double* x, int32_t icol) {
  double s = 0.0;
  if (P->dynamics == ORC_UNICYCLE) {
    for (int i = 0; i < 3; ++i) s += P->Qf[i] * (x[i] - P->goal[i]) * (x[i] - P->goal[i]);
  } else {
    if (P->flags & ORC_FLAG_POSE_COST) {
      s += pose_terms(P, x, P->Qf, icol);
    } else {
      double org[7][3];
      orc_arm_frames(x, P->dh, org, NULL);
      s += P->Qf[0] * sqdist(org[6], P->goal, 3);
    }
    s += limit_penalty(P, x);
  }
  return s;
}

/* Task-space position p(x): planar position, or end-effector position. */
static void task_point(const orc_problem* P, const double* x, double* pt) {
  if (P->dynamics == ORC_UNICYCLE) {
    pt[0] = x[0];
    pt[1] = x[1];
  } else {
    double org[7][3];
    orc_arm_frames(x, P->dh, org, NULL);
    pt[0] = org[6][0];
    pt[1] = org[6][1];
    pt[2] = org[6][2];
  }
}

/* Collision test of one state against every obstacle (Sec. II-B.1), the
 * obstacles displaced by tj * vel (vel NULL: frozen).  Returns the lowest
 * obstacle index in contact, or -1; lowers *clear to the smallest relative
 * distance to a contact boundary seen. */
static int32_t state_contact(const orc_problem* P, const double* x, const double* obs,
                             const double* vel, int32_t n_obs, double tj, double* clear) {
  int32_t hit = -1;
  if (P->dynamics == ORC_UNICYCLE) {
    for (int32_t i = 0; i < n_obs; ++i) {
      double o[2] = {obs[3 * i], obs[3 * i + 1]};
      if (vel) {
        o[0] += tj * vel[2 * i];
        o[1] += tj * vel[2 * i + 1];
      }
      double R = P->robot_radius + obs[3 * i + 2];
      double d2 = sqdist(x, o, 2);
      double c = fabs(sqrt(d2) - R) / (R > 0.0 ? R : 1.0);
      if (c < *clear) *clear = c;
      if (hit < 0 && d2 <= R * R) hit = i;
    }
  } else {
    double org[7][3];
    double cen[3 * 64];
    orc_arm_frames(x, P->dh, org, NULL);
    orc_arm_spheres(org, P->n_link_spheres, cen);
    for (int32_t i = 0; i < n_obs; ++i) {
      double o[3] = {obs[4 * i], obs[4 * i + 1], obs[4 * i + 2]};
      if (vel)
        for (int c = 0; c < 3; ++c) o[c] += tj * vel[3 * i + c];
      for (int32_t s = 0; s < P->n_link_spheres; ++s) {
        double R = P->link_sphere_radius + obs[4 * i + 3];
        double d2 = sqdist(cen + 3 * s, o, 3);
        double c = fabs(sqrt(d2) - R) / (R > 0.0 ? R : 1.0);
        if (c < *clear) *clear = c;
        if (hit < 0 && d2 <= R * R) hit = i;
      }
    }
  }
  return hit;
}

/* dynamics step x_{j+1} = f(x_j, u_j) (Eq. (4)) */
static void step_dynamics(const orc_problem* P, const double* x, const double* u, double* xn) {
  if (P->dynamics == ORC_UNICYCLE) {
    orc_unicycle_step(x, u, P->dt, xn);
  } else {
    /* joint-velocity command: q <- q + u dt, qdot <- u (Sec. III-C) */
    for (int i = 0; i < 6; ++i) {
      xn[i] = x[i] + u[i] * P->dt;
      xn[6 + i] = u[i];
    }
  }
}

/* One rollout: Alg. 1 "simulate", cost Eq. (5), collision indicator and the
 * first contact (Sec. II-B.1), tested on x_1..x_N.  With the pose cost the
 * stage and terminal terms also count I_col(x_j) for j = 0..N, and x_0
 * enters the boundary clearance. */
void orc_simulate_moving(const orc_problem* P, const double* x0, const double* ut,
                         const double* obs, const double* vel, int32_t n_obs, double* traj,
                         double* S, int32_t* col, int32_t* first_obs, double* p_term,
                         double* p_first, double* clearance) {
  int32_t n, m, p;
  orc_dims(P->dynamics, &n, &m, &p);
  const int pose = P->dynamics == ORC_ARM6 && (P->flags & ORC_FLAG_POSE_COST);
  double x[12], xn[12];
  memcpy(x, x0, sizeof(double) * (size_t)n);
  if (traj) memcpy(traj, x, sizeof(double) * (size_t)n);
  double cost = 0.0, clear = INFINITY;
  int32_t c = 0, f = -1;
  double pf[3] = {0.0, 0.0, 0.0};
  int32_t icol = pose ? (state_contact(P, x, obs, vel, n_obs, 0.0, &clear) >= 0) : 0;
  for (int32_t j = 0; j < P->N; ++j) {
    cost += stage_cost(P, x, ut + j * m, icol);
    step_dynamics(P, x, ut + j * m, xn);
    memcpy(x, xn, sizeof(double) * (size_t)n);
    if (traj) memcpy(traj + (size_t)(j + 1) * n, x, sizeof(double) * (size_t)n);
    int32_t hit = state_contact(P, x, obs, vel, n_obs, (double)(j + 1) * P->dt, &clear);
    icol = hit >= 0;
    if (hit >= 0 && !c) {
      c = 1;
      f = hit;
      task_point(P, x, pf);
    }
  }
  cost += terminal_cost(P, x, icol);
  *S = cost;
  *col = c;
  *first_obs = f;
  task_point(P, x, p_term);
  for (int32_t i = 0; i < p; ++i) p_first[i] = pf[i];
  if (clearance) *clearance = clear;
}

void orc_simulate(const orc_problem* P, const double* x0, const double* ut, const double* obs,
                  int32_t n_obs, double* traj, double* S, int32_t* col, int32_t* first_obs,
                  double* p_term, double* p_first, double* clearance) {
  orc_simulate_moving(P, x0, ut, obs, NULL, n_obs, traj, S, col, first_obs, p_term, p_first,
                      clearance);
}

/* Surface clearance of obstacle i from the robot at x0: distance to the
 * centre minus the obstacle radius (for the arm, the minimum over the link
 * spheres of the distance to their centres). */
static double clearance_of(const orc_problem* P, const double* x0, const double* obs, int32_t i) {
  if (P->dynamics == ORC_UNICYCLE) return sqrt(sqdist(x0, obs + 3 * i, 2)) - obs[3 * i + 2];
  double org[7][3];
  double cen[3 * 64];
  orc_arm_frames(x0, P->dh, org, NULL);
  orc_arm_spheres(org, P->n_link_spheres, cen);
  double ci = INFINITY;
  for (int32_t s = 0; s < P->n_link_spheres; ++s) {
    double c = sqrt(sqdist(cen + 3 * s, obs + 4 * i, 3)) - obs[4 * i + 3];
    if (c < ci) ci = c;
  }
  return ci;
}

/* Closest obstacle o* to the current robot (the reference obstacle of
 * Sec. I and Sec. II-B.2): smallest surface clearance, ties to the lowest
 * index.  *margin (may be NULL) receives the second-smallest clearance minus
 * the smallest (INFINITY with fewer than two obstacles). */
int32_t orc_closest_obstacle_margin(const orc_problem* P, const double* x0, const double* obs,
                                    int32_t n_obs, double* margin) {
  int32_t best = -1;
  double bestc = INFINITY, second = INFINITY;
  for (int32_t i = 0; i < n_obs; ++i) {
    double c = clearance_of(P, x0, obs, i);
    if (best < 0 || c < bestc) {
      second = bestc;
      best = i;
      bestc = c;
    } else if (c < second) {
      second = c;
    }
  }
  if (margin) *margin = n_obs > 1 ? second - bestc : INFINITY;
  return best;
}

int32_t orc_closest_obstacle(const orc_problem* P, const double* x0, const double* obs, int32_t n_obs) {
  return orc_closest_obstacle_margin(P, x0, obs, n_obs, NULL);
}

/* Obstacle velocity, Sec. II-B.3, Eq. (17): the mean of the H'-1 finite
 * differences of the newest H' = min(H, h_avail) observations. */
void orc_obstacle_velocity(const double* hist, int32_t h_avail, int32_t n_obs, int32_t p, int32_t idx,
                           int32_t H, double dt, double v[3]) {
  int32_t Hp = h_avail < H ? h_avail : H;
  v[0] = v[1] = v[2] = 0.0;
  if (Hp < 2) return;
  for (int32_t h = 0; h <= Hp - 2; ++h) {
    const double* o_new = hist + ((size_t)h * n_obs + idx) * p;
    const double* o_old = hist + ((size_t)(h + 1) * n_obs + idx) * p;
    for (int32_t i = 0; i < p; ++i) v[i] += (o_new[i] - o_old[i]) / dt;
  }
  for (int32_t i = 0; i < p; ++i) v[i] /= (double)(Hp - 1);
}

/* ------------------------------------------------------------------ */
/* DBSCAN (Sec. II-B.2), by its definition                            */
/* ------------------------------------------------------------------ */

/* Neighbourhood N(k) = {l : |z_k - z_l| <= eps} (k itself included); core
 * iff |N(k)| >= min_pts; clusters are the connected components of the
 * core points under the neighbour relation, found here by breadth-first
 * search from the cores in ascending index order, so cluster c is the one
 * whose lowest core index is the c-th smallest; a non-core point with a
 * core neighbour joins the cluster of its lowest-index core neighbour;
 * everything else is noise (-1).  Returns the number of clusters. */
static int32_t within(const double* a, const double* b, int32_t p, double r2) {
  return sqdist(a, b, p) <= r2 ? 1 : 0;
}

int32_t orc_dbscan(const double* z, int32_t V, int32_t p, double eps, int32_t min_pts,
                   int32_t* ncount, int32_t* core, int32_t* label) {
  const double r2 = eps * eps;
  for (int32_t k = 0; k < V; ++k) {
    int32_t c = 0;
    for (int32_t l = 0; l < V; ++l) c += within(z + (size_t)k * p, z + (size_t)l * p, p, r2);
    ncount[k] = c;
    core[k] = c >= min_pts ? 1 : 0;
    label[k] = -1;
  }
  int32_t* queue = (int32_t*)malloc(sizeof(int32_t) * (size_t)(V > 0 ? V : 1));
  int32_t M = 0;
  for (int32_t k = 0; k < V; ++k) {
    if (!core[k] || label[k] >= 0) continue;
    int32_t head = 0, tail = 0;
    label[k] = M;
    queue[tail++] = k;
    while (head < tail) {
      int32_t a = queue[head++];
      for (int32_t l = 0; l < V; ++l) {
        if (core[l] && label[l] < 0 && within(z + (size_t)a * p, z + (size_t)l * p, p, r2)) {
          label[l] = M;
          queue[tail++] = l;
        }
      }
    }
    ++M;
  }
  free(queue);
  for (int32_t k = 0; k < V; ++k) {
    if (core[k]) continue;
    for (int32_t l = 0; l < V; ++l) {
      if (core[l] && within(z + (size_t)k * p, z + (size_t)l * p, p, r2)) {
        label[k] = label[l];
        break;
      }
    }
  }
  return M;
}

/* ------------------------------------------------------------------ */
/* Path-integral update, Eq. (6)-(7) and Eq. (19)-(20)                 */
/* ------------------------------------------------------------------ */

/* Weights exp(-S/lambda) normalised over the rollouts in `set`, evaluated
 * as exp(-(S - S_min)/lambda) (the common factor cancels), and
 * U_new = U + sum_k w_k eps_k. */
void orc_weighted_update(int32_t n_set, const int32_t* set, const double* S, const double* eps_eff,
                         int32_t N, int32_t m, double lambda, const double* U, double* U_new,
                         double* weight_out, double* s_min) {
  double smin = INFINITY;
  for (int32_t a = 0; a < n_set; ++a)
    if (S[set[a]] < smin) smin = S[set[a]];
  double* w = (double*)malloc(sizeof(double) * (size_t)(n_set > 0 ? n_set : 1));
  double wsum = 0.0;
  for (int32_t a = 0; a < n_set; ++a) {
    w[a] = exp(-(S[set[a]] - smin) / lambda);
    wsum += w[a];
  }
  for (int32_t e = 0; e < N * m; ++e) {
    double acc = 0.0;
    for (int32_t a = 0; a < n_set; ++a) acc += (w[a] / wsum) * eps_eff[(size_t)set[a] * N * m + e];
    U_new[e] = U[e] + acc;
  }
  if (weight_out)
    for (int32_t a = 0; a < n_set; ++a) weight_out[set[a]] = w[a] / wsum;
  if (s_min) *s_min = smin;
  free(w);
}

/* ------------------------------------------------------------------ */
/* Cluster statistics and selection, Alg. 1 [Cluster stats] and        */
/* [Selection], Eq. (14)-(18)                                          */
/* ------------------------------------------------------------------ */

/* On the labels of the nV feasible rollouts (0..M-1, -1 noise; M >= 1) with
 * their costs S_v and unit terminal displacements g ([nV][p], Eq. (15)):
 * per cluster the size, the mean cost (Alg. 1) and the normalised mean
 * direction (Eq. (16)); then the cluster of minimum mean cost (Eq. (14)), or,
 * in a dynamic scene whose closest obstacle has a usable velocity estimate
 * (Eq. (17)), the cluster whose direction has the smallest dot product with
 * the obstacle's normalised velocity (Eq. (18)).  Ties go to the lowest
 * label.  Fills the cluster arrays, selected, selected_size, rule, h_used,
 * margin, v_obs, v_obs_hat and the DYN_STATIC status bit of *out; returns the
 * selected label. */
int32_t orc_select_cluster(const orc_problem* P, int32_t nV, const int32_t* lab, int32_t M,
                           const double* S_v, const double* g, const double* hist, int32_t h_avail,
                           int32_t n_obs, int32_t closest, orc_out* out) {
  int32_t n, m, p;
  orc_dims(P->dynamics, &n, &m, &p);
  double* mc = (double*)calloc((size_t)M, sizeof(double));
  double* vd = (double*)calloc((size_t)M * 3, sizeof(double));
  int32_t* sz = (int32_t*)calloc((size_t)M, sizeof(int32_t));
  for (int32_t a = 0; a < nV; ++a) {
    int32_t c = lab[a];
    if (c < 0) continue;
    mc[c] += S_v[a];
    for (int32_t i = 0; i < p; ++i) vd[(size_t)c * 3 + i] += g[(size_t)a * p + i];
    sz[c] += 1;
  }
  for (int32_t c = 0; c < M; ++c) {
    mc[c] /= (double)sz[c];
    double nv = 0.0;
    for (int32_t i = 0; i < p; ++i) {
      vd[(size_t)c * 3 + i] /= (double)sz[c];
      nv += vd[(size_t)c * 3 + i] * vd[(size_t)c * 3 + i];
    }
    nv = sqrt(nv);
    for (int32_t i = 0; i < p; ++i) vd[(size_t)c * 3 + i] /= (nv + P->norm_eps);
  }

  int32_t rule = ORC_STATIC;
  double vhat[3] = {0.0, 0.0, 0.0};
  if (P->scene_mode == ORC_DYNAMIC) {
    int32_t Hp = h_avail < P->history_len ? h_avail : P->history_len;
    out->h_used = Hp;
    double v[3] = {0.0, 0.0, 0.0};
    if (closest >= 0)
      orc_obstacle_velocity(hist, h_avail, n_obs, p, closest, P->history_len, P->dt, v);
    double nv = 0.0;
    for (int32_t i = 0; i < p; ++i) nv += v[i] * v[i];
    nv = sqrt(nv);
    for (int32_t i = 0; i < p; ++i) {
      out->v_obs[i] = v[i];
      vhat[i] = v[i] / (nv + P->norm_eps);
      out->v_obs_hat[i] = vhat[i];
    }
    if (Hp >= 2 && closest >= 0 && !(nv < P->v_obs_min)) rule = ORC_DYNAMIC;
    else out->status |= ORC_ST_DYN_STATIC;
  }
  out->rule = rule;
  int32_t best = 0;
  double kbest = INFINITY, second = INFINITY;
  for (int32_t c = 0; c < M; ++c) {
    double key = 0.0;
    if (rule == ORC_STATIC) {
      key = mc[c];
    } else {
      for (int32_t i = 0; i < p; ++i) key += vd[(size_t)c * 3 + i] * vhat[i];
    }
    if (c == 0 || key < kbest) {
      if (c > 0) second = kbest;
      kbest = key;
      best = c;
    } else if (key < second) {
      second = key;
    }
  }
  out->margin = M > 1 ? second - kbest : INFINITY;
  out->selected = best;
  out->selected_size = sz[best];
  int32_t cap = out->c_cap < M ? out->c_cap : M;
  for (int32_t c = 0; c < cap; ++c) {
    if (out->c_mean_cost) out->c_mean_cost[c] = mc[c];
    if (out->c_size) out->c_size[c] = sz[c];
    if (out->c_dir)
      for (int32_t i = 0; i < p; ++i) out->c_dir[(size_t)c * p + i] = vd[(size_t)c * 3 + i];
  }
  free(mc);
  free(vd);
  free(sz);
  return best;
}

/* ------------------------------------------------------------------ */
/* Alg. 1                                                              */
/* ------------------------------------------------------------------ */

static int32_t all_finite(const double* a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(a[i])) return 0;
  return 1;
}

/* Alg. 1 from [Pruning] on, given the rollout records (cost, collision
 * indicator, first obstacle hit, terminal and first-contact points, applied
 * perturbations). */
static void post_rollouts(const orc_problem* P, const double* x_t, const double* U, const double* obs,
                          int32_t n_obs, const double* hist, int32_t h_avail, const double* S,
                          const int32_t* col, const int32_t* fo, const double* pT, const double* pF,
                          const double* E, orc_out* out) {
  int32_t n, m, p;
  orc_dims(P->dynamics, &n, &m, &p);
  const int32_t N = P->N, K = P->K, NM = P->N * m;
  /* [Pruning] Eq. (9)-(10) */
  int32_t* Vi = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
  int32_t nV = 0, nC = 0;
  for (int32_t k = 0; k < K; ++k) {
    if (col[k]) ++nC;
    else Vi[nV++] = k;
  }
  out->n_col = nC;
  out->n_feas = nV;
  {
    double cm = INFINITY;
    int32_t c = orc_closest_obstacle_margin(P, x_t, obs, n_obs, &cm);
    out->closest_margin = cm;
    out->closest = out->closest_force >= -1 ? out->closest_force : c;
  }

  int32_t* set = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
  int32_t n_set = 0;
  double* z = NULL;
  double* g = NULL;
  int32_t* lab = NULL;

  if (nC == 0 || nV == 0) {
    /* [Fallback] Eq. (6)-(7) over every rollout */
    out->branch = nC == 0 ? ORC_BRANCH_FALLBACK : ORC_BRANCH_ALL_COLLIDE;
    out->status |= nC == 0 ? ORC_ST_FALLBACK : ORC_ST_ALL_COLLIDE;
    for (int32_t k = 0; k < K; ++k) set[n_set++] = k;
  } else {
    out->branch = ORC_BRANCH_CLUSTER;
    /* reference point, Eq. (11), restricted to the rollouts whose first
     * contact is the closest obstacle when there are any */
    int32_t nA = 0;
    for (int32_t k = 0; k < K; ++k)
      if (col[k] && fo[k] == out->closest) ++nA;
    int32_t use_all = nA == 0;
    const double* src = P->ref_mode == ORC_REF_FIRST_CONTACT ? pF : pT;
    double ref[3] = {0.0, 0.0, 0.0};
    int32_t cnt = 0;
    for (int32_t k = 0; k < K; ++k) {
      if (!col[k]) continue;
      if (!use_all && fo[k] != out->closest) continue;
      for (int32_t i = 0; i < p; ++i) ref[i] += src[(size_t)k * p + i];
      ++cnt;
    }
    for (int32_t i = 0; i < p; ++i) ref[i] /= (double)cnt;
    out->n_ref = cnt;
    for (int32_t i = 0; i < p; ++i) out->ref_point[i] = ref[i];

    /* features, Eq. (12)-(13), and unit terminal displacement, Eq. (15) */
    double p0[3];
    task_point(P, x_t, p0);
    z = (double*)malloc(sizeof(double) * (size_t)nV * p);
    g = (double*)malloc(sizeof(double) * (size_t)nV * p);
    for (int32_t a = 0; a < nV; ++a) {
      const double* pk = pT + (size_t)Vi[a] * p;
      double d[3], nd = 0.0, e[3], ne = 0.0;
      for (int32_t i = 0; i < p; ++i) {
        d[i] = pk[i] - ref[i];
        nd += d[i] * d[i];
        e[i] = pk[i] - p0[i];
        ne += e[i] * e[i];
      }
      nd = sqrt(nd);
      ne = sqrt(ne);
      for (int32_t i = 0; i < p; ++i) {
        z[(size_t)a * p + i] = d[i] / (nd + P->norm_eps);
        g[(size_t)a * p + i] = e[i] / (ne + P->norm_eps);
      }
    }

    /* DBSCAN on the features of the feasible rollouts */
    int32_t* cnt_n = (int32_t*)malloc(sizeof(int32_t) * (size_t)nV);
    int32_t* cor = (int32_t*)malloc(sizeof(int32_t) * (size_t)nV);
    lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)nV);
    int32_t M = orc_dbscan(z, nV, p, P->dbscan_eps, P->dbscan_min_pts, cnt_n, cor, lab);
    out->n_clusters = M;
    if (out->ncount) memcpy(out->ncount, cnt_n, sizeof(int32_t) * (size_t)nV);
    if (out->core) memcpy(out->core, cor, sizeof(int32_t) * (size_t)nV);
    free(cnt_n);
    free(cor);

    if (M == 0) {
      out->status |= ORC_ST_NO_CLUSTER;
      for (int32_t a = 0; a < nV; ++a) set[n_set++] = Vi[a];
    } else {
      double* Sv = (double*)malloc(sizeof(double) * (size_t)nV);
      for (int32_t a = 0; a < nV; ++a) Sv[a] = S[Vi[a]];
      int32_t best = orc_select_cluster(P, nV, lab, M, Sv, g, hist, h_avail, n_obs, out->closest, out);
      free(Sv);
      for (int32_t a = 0; a < nV; ++a)
        if (lab[a] == best) set[n_set++] = Vi[a];
    }
  }

  /* [Within-cluster weighting] + [Update], Eq. (19)-(20) (Eq. (6)-(7) on the
   * fallback branches) */
  double* Un = (double*)malloc(sizeof(double) * (size_t)NM);
  double* wfull = NULL;
  if (out->weight) {
    memset(out->weight, 0, sizeof(double) * (size_t)K);
    wfull = out->weight;
  }
  orc_weighted_update(n_set, set, S, E, N, m, P->lambda, U, Un, wfull, &out->s_min);

  /* [Execute] apply u_t; shift and warm-start (last control repeated) */
  if (out->U_new) memcpy(out->U_new, Un, sizeof(double) * (size_t)NM);
  if (out->u_out) memcpy(out->u_out, Un, sizeof(double) * (size_t)m);
  if (out->U_next) {
    for (int32_t j = 0; j < N; ++j) {
      int32_t src = j + 1 < N ? j + 1 : N - 1;
      memcpy(out->U_next + (size_t)j * m, Un + (size_t)src * m, sizeof(double) * (size_t)m);
    }
  }

  if (out->v_idx) memcpy(out->v_idx, Vi, sizeof(int32_t) * (size_t)nV);
  if (out->z && z) memcpy(out->z, z, sizeof(double) * (size_t)nV * p);
  if (out->g && g) memcpy(out->g, g, sizeof(double) * (size_t)nV * p);
  if (out->label && lab) memcpy(out->label, lab, sizeof(int32_t) * (size_t)nV);
  free(Un);
  free(z);
  free(g);
  free(lab);
  free(set);
  free(Vi);
}

static void init_out(orc_out* out) {
  out->branch = ORC_BRANCH_FALLBACK;
  out->n_col = out->n_feas = out->n_ref = out->n_clusters = 0;
  out->selected = -1;
  out->selected_size = 0;
  out->closest = -1;
  out->rule = ORC_STATIC;
  out->h_used = 0;
  out->status = 0;
  out->margin = INFINITY;
  out->closest_margin = INFINITY;
  out->s_min = 0.0;
  for (int i = 0; i < 3; ++i) out->ref_point[i] = out->v_obs[i] = out->v_obs_hat[i] = 0.0;
}

int32_t orc_replan(const orc_problem* P, const double* x_t, const double* U, const double* obs,
                   int32_t n_obs, const double* hist, int32_t h_avail, uint32_t step, orc_out* out) {
  int32_t n, m, p;
  if (orc_dims(P->dynamics, &n, &m, &p) != 0) return -1;
  const int32_t N = P->N, K = P->K, NM = P->N * m;
  if (N < 1 || K < 1 || !(P->lambda > 0.0) || n_obs < 0 || n_obs > ORC_MAX_OBS) return -1;

  init_out(out);

  /* non-finite input: no update, no shift */
  if (!all_finite(x_t, (size_t)n) || !all_finite(obs, (size_t)n_obs * (p + 1))) {
    out->status = ORC_ST_NONFINITE;
    if (out->U_new) memcpy(out->U_new, U, sizeof(double) * (size_t)NM);
    if (out->U_next) memcpy(out->U_next, U, sizeof(double) * (size_t)NM);
    if (out->u_out) memcpy(out->u_out, U, sizeof(double) * (size_t)m);
    return 0;
  }

  double* S = (double*)malloc(sizeof(double) * (size_t)K);
  int32_t* col = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
  int32_t* fo = (int32_t*)malloc(sizeof(int32_t) * (size_t)K);
  double* pT = (double*)malloc(sizeof(double) * (size_t)K * p);
  double* pF = (double*)malloc(sizeof(double) * (size_t)K * p);
  double* E = (double*)malloc(sizeof(double) * (size_t)K * NM);
  double* eps = (double*)malloc(sizeof(double) * (size_t)NM);
  double* ut = (double*)malloc(sizeof(double) * (size_t)NM);

  /* constant-velocity obstacles: each obstacle's own velocity by Eq. (17) */
  double* vel = NULL;
  if ((P->flags & ORC_FLAG_OBS_CONST_VEL) && n_obs > 0) {
    vel = (double*)malloc(sizeof(double) * (size_t)n_obs * p);
    for (int32_t i = 0; i < n_obs; ++i) {
      double v[3];
      orc_obstacle_velocity(hist, h_avail, n_obs, p, i, P->history_len, P->dt, v);
      for (int32_t d = 0; d < p; ++d) vel[(size_t)i * p + d] = v[d];
    }
  }

  /* [Rollouts] Alg. 1: sample, perturb (Eq. (3)), simulate (Eq. (4)),
   * cost (Eq. (5)), collision indicator. */
  for (int32_t k = 0; k < K; ++k) {
    orc_rollout_noise(P, step, k, NULL, eps);
    for (int32_t j = 0; j < N; ++j)
      for (int32_t i = 0; i < m; ++i) {
        double u = U[j * m + i] + eps[j * m + i];
        if (u < P->u_min[i]) u = P->u_min[i];
        if (u > P->u_max[i]) u = P->u_max[i];
        ut[j * m + i] = u;
        E[(size_t)k * NM + j * m + i] = u - U[j * m + i];
      }
    double clear;
    orc_simulate_moving(P, x_t, ut, obs, vel, n_obs, NULL, &S[k], &col[k], &fo[k],
                        pT + (size_t)k * p, pF + (size_t)k * p, &clear);
    if (out->clearance) out->clearance[k] = clear;
  }

  post_rollouts(P, x_t, U, obs, n_obs, hist, h_avail, S, col, fo, pT, pF, E, out);
  if (out->S) memcpy(out->S, S, sizeof(double) * (size_t)K);
  if (out->col) memcpy(out->col, col, sizeof(int32_t) * (size_t)K);
  if (out->first_obs) memcpy(out->first_obs, fo, sizeof(int32_t) * (size_t)K);
  if (out->p_term) memcpy(out->p_term, pT, sizeof(double) * (size_t)K * p);
  if (out->p_first) memcpy(out->p_first, pF, sizeof(double) * (size_t)K * p);
  if (out->eps_eff) memcpy(out->eps_eff, E, sizeof(double) * (size_t)K * NM);

  free(S);
  free(col);
  free(fo);
  free(pT);
  free(pF);
  free(E);
  free(eps);
  free(ut);
  free(vel);
  return 0;
}

int32_t orc_replan_from_rollouts(const orc_problem* P, const double* x_t, const double* U,
                                 const double* obs, int32_t n_obs, const double* hist,
                                 int32_t h_avail, const double* S, const int32_t* col,
                                 const int32_t* first_obs, const double* p_term,
                                 const double* p_first, const double* eps_eff, orc_out* out) {
  int32_t n, m, p;
  if (orc_dims(P->dynamics, &n, &m, &p) != 0) return -1;
  if (P->N < 1 || P->K < 1 || !(P->lambda > 0.0) || n_obs < 0 || n_obs > ORC_MAX_OBS) return -1;
  init_out(out);
  post_rollouts(P, x_t, U, obs, n_obs, hist, h_avail, S, col, first_obs, p_term, p_first, eps_eff,
                out);
  return 0;
}
