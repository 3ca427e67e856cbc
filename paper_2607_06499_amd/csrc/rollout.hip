// rollout.hip -- noise, forward simulation, cost and collision of every
// rollout (Alg. 1 [Rollouts], Eq. (3)-(5), Sec. II-B.1).  Each block also
// leaves a partial record (counts and sums for pruning and the reference
// point of Eq. (9)-(11)); the next kernel reduces those records.
//
// Layout: one rollout per 64-lane segment of a wavefront (two per wave when
// the N+1 states fit in 32 lanes).  Lane j of a segment owns control u_j and
// state x_j: the noise of a step is drawn in its lane, the linear parts of the
// dynamics are prefix sums across lanes (the heading of the unicycle, the joint
// angles of the arm), and every lane evaluates its own stage cost, collision
// test and (arm) forward kinematics.  The serial N-step recursion of Eq. (4)
// thus becomes log2(N) shuffle steps and all work of a step runs in parallel.
#include "device.hpp"
#include "launch.hpp"

namespace cemppi {

// ---------------------------------------------------------------------------
// shared prologue: obstacles into LDS, finiteness, closest obstacle o*.
struct ObsLds {
  float4 o[kMaxObs];     // (x, y, z, R^2) with R = robot/sphere radius + obstacle radius
  float r[kMaxObs];      // obstacle radius
  float4 v[kMaxObs];     // obstacle velocity (constant-velocity obstacles; else 0)
  float4 live[kMaxObs];  // the obstacles a rollout can reach, in index order
  float4 vlive[kMaxObs]; // their velocities
  int idx[kMaxObs];      // their obstacle indices
  int n_live;
};

// Arm forward kinematics: origins P0..P6 of the standard DH chain
// (A_i = Rz(q_i + off_i) Tz(d_i) Tx(a_i) Rx(alpha_i)); P6 is p_ee(q).
__device__ __forceinline__ void arm_origins(const Cfg& c, const float* q, float P[7][3],
                                            float* Re = nullptr) {
  float r00 = 1.f, r01 = 0.f, r02 = 0.f, r10 = 0.f, r11 = 1.f, r12 = 0.f, r20 = 0.f, r21 = 0.f,
        r22 = 1.f;
  float tx = 0.f, ty = 0.f, tz = 0.f;
  P[0][0] = P[0][1] = P[0][2] = 0.f;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float st, ct;
    sincosf(q[i] + c.dh_off[i], &st, &ct);
    const float ca = c.dh_ca[i], sa = c.dh_sa[i], a = c.dh_a[i], d = c.dh_d[i];
    // translation of frame i in frame i-1: (a cos th, a sin th, d)
    const float lx = a * ct, ly = a * st, lz = d;
    tx += r00 * lx + r01 * ly + r02 * lz;
    ty += r10 * lx + r11 * ly + r12 * lz;
    tz += r20 * lx + r21 * ly + r22 * lz;
    // rotation Rz(th) Rx(alpha)
    const float a00 = ct, a01 = -st * ca, a02 = st * sa;
    const float a10 = st, a11 = ct * ca, a12 = -ct * sa;
    const float a21 = sa, a22 = ca;
    const float n00 = r00 * a00 + r01 * a10, n01 = r00 * a01 + r01 * a11 + r02 * a21,
                n02 = r00 * a02 + r01 * a12 + r02 * a22;
    const float n10 = r10 * a00 + r11 * a10, n11 = r10 * a01 + r11 * a11 + r12 * a21,
                n12 = r10 * a02 + r11 * a12 + r12 * a22;
    const float n20 = r20 * a00 + r21 * a10, n21 = r20 * a01 + r21 * a11 + r22 * a21,
                n22 = r20 * a02 + r21 * a12 + r22 * a22;
    r00 = n00; r01 = n01; r02 = n02;
    r10 = n10; r11 = n11; r12 = n12;
    r20 = n20; r21 = n21; r22 = n22;
    P[i + 1][0] = tx;
    P[i + 1][1] = ty;
    P[i + 1][2] = tz;
  }
  if (Re) {
    Re[0] = r00; Re[1] = r01; Re[2] = r02;
    Re[3] = r10; Re[4] = r11; Re[5] = r12;
    Re[6] = r20; Re[7] = r21; Re[8] = r22;
  }
}

// Orientation error of the pose cost (Sec. III-C): the angle of the relative
// rotation R_g^T R_ee, atan2(|v|, tr - 1) with tr its trace and v its
// antisymmetric part (|v| = 2 sin, tr - 1 = 2 cos); well conditioned at every
// angle in [0, pi].
__device__ __forceinline__ float rot_angle(const Cfg& c, const float* Re) {
  float tr = 0.f, vx = 0.f, vy = 0.f, vz = 0.f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float g0 = c.Rg[3 * i], g1 = c.Rg[3 * i + 1], g2 = c.Rg[3 * i + 2];
    const float e0 = Re[3 * i], e1 = Re[3 * i + 1], e2 = Re[3 * i + 2];
    tr += g0 * e0 + g1 * e1 + g2 * e2;
    vx += g2 * e1 - g1 * e2;
    vy += g0 * e2 - g2 * e0;
    vz += g1 * e0 - g0 * e1;
  }
  return atan2f(sqrtf(vx * vx + vy * vy + vz * vz), tr - 1.f);
}

__device__ __forceinline__ void sphere_centre(const Cfg& c, const float P[7][3], int s, float& x,
                                              float& y, float& zz) {
  // the segment of sphere s is a kernel argument, so this switch is a
  // wave-uniform (scalar) branch
  const int sg = c.sph_seg[s];
  float ax, ay, az, bx, by, bz;
  switch (sg) {
#define CEMPPI_SEG(i)                                     \
  case i:                                                 \
    ax = P[i][0]; ay = P[i][1]; az = P[i][2];             \
    bx = P[i + 1][0]; by = P[i + 1][1]; bz = P[i + 1][2]; \
    break;
    CEMPPI_SEG(0)
    CEMPPI_SEG(1)
    CEMPPI_SEG(2)
    CEMPPI_SEG(3)
    CEMPPI_SEG(4)
    default:
      ax = P[5][0]; ay = P[5][1]; az = P[5][2];
      bx = P[6][0]; by = P[6][1]; bz = P[6][2];
      break;
#undef CEMPPI_SEG
  }
  const float t = c.sph_t[s];
  x = ax + t * (bx - ax);
  y = ay + t * (by - ay);
  zz = az + t * (bz - az);
}

__device__ __forceinline__ float limit_penalty(const Cfg& c, const float* q) {
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float e = fabsf(q[i]) - c.qlim[i];
    s += e > 0.f ? e * e : 0.f;
  }
  return c.wlim * s;
}

// Prologue run by every block: stages the obstacles, checks the inputs and
// computes o* (smallest surface clearance, ties to the lowest index) and
// p(x_t).  Returns through LDS: s_bad, s_closest, s_p0.
// CVM: constant-velocity obstacles never (0), always (1) or as c.cv says (2).
// Arm (DYN 1): *s_c0 receives the state part of the stage cost of x_t
// (with the pose cost, including its contact indicator).
template <int DYN, int CVM = 2>
__device__ void prologue(const Cfg& c, const Bufs& b, const float* __restrict__ x_t,
                         const float* __restrict__ obs, int n_obs, ObsLds& L, int& s_bad,
                         int& s_closest, float* s_p0, float* s_c0 = nullptr) {
  const int tid = threadIdx.x;
  const int P = DYN == 0 ? 2 : 3;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  if (tid < n_obs) {
    const float* o = obs + tid * (P + 1);
    float ok = 1.f;
    for (int i = 0; i <= P; ++i) ok = isfinite(o[i]) ? ok : 0.f;
    if (ok == 0.f) atomicOr(&s_bad, 1);
    const float R = (DYN == 0 ? c.robot_r : c.rs) + o[P];
    L.o[tid] = make_float4(o[0], o[1], DYN == 0 ? 0.f : o[2], R * R);
    L.r[tid] = o[P];
    // constant-velocity obstacles: Eq. (17) for every obstacle over the ring
    // as it will be after this replan's push (the current observation is the
    // newest entry), telescoped to (o_t - o_{t-H'+1}) / ((H' - 1) dt)
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (CVM == 2 ? c.cv != 0 : CVM == 1) {
      const Ctrl* ct = b.ctrl;
      const int cnt = (ct->hs_nobs == n_obs ? ct->hs_count : 0) + 1;
      const int Hp = cnt < c.H ? cnt : c.H;
      if (Hp >= 2) {
        const int h1 = (ct->hs_head - (Hp - 2) + 2 * c.H) % c.H;
        const float* old = b.hist + ((size_t)h1 * c.max_obs + tid) * P;
        const float den = (float)(Hp - 1) * c.dt;
        v.x = (o[0] - old[0]) / den;
        v.y = (o[1] - old[1]) / den;
        if (DYN != 0) v.z = (o[2] - old[2]) / den;
      }
    }
    L.v[tid] = v;
  }
  if (tid < c.n && !isfinite(x_t[tid])) atomicOr(&s_bad, 1);
  __syncthreads();
  if (tid < kWave) {
    float cl = INFINITY;
    int idx = kInt32Max;
    if (DYN == 0) {
      const float x0 = x_t[0], y0 = x_t[1];
      if (tid == 0) {
        s_p0[0] = x0;
        s_p0[1] = y0;
        s_p0[2] = 0.f;
      }
      if (tid < n_obs) {
        cl = sqrtf(dist2_2(x0, y0, L.o[tid].x, L.o[tid].y)) - L.r[tid];
        idx = tid;
      }
    } else {
      float q[6], Pm[7][3], Re[9];
      for (int i = 0; i < 6; ++i) q[i] = x_t[i];
      arm_origins(c, q, Pm, Re);
      if (tid == 0) {
        s_p0[0] = Pm[6][0];
        s_p0[1] = Pm[6][1];
        s_p0[2] = Pm[6][2];
      }
      bool touch = false;
      if (tid < n_obs) {
        for (int s = 0; s < c.ns; ++s) {
          float sx, sy, sz;
          sphere_centre(c, Pm, s, sx, sy, sz);
          const float d2 = dist2_3(sx, sy, sz, L.o[tid].x, L.o[tid].y, L.o[tid].z);
          const float v = sqrtf(d2) - L.r[tid];
          cl = v < cl ? v : cl;
          touch |= d2 <= L.o[tid].w;
        }
        idx = tid;
      }
      const bool icol0 = __ballot(touch) != 0ull;
      if (tid == 0 && s_c0) {
        const float d2g = sq(Pm[6][0] - c.goal[0]) + sq(Pm[6][1] - c.goal[1]) + sq(Pm[6][2] - c.goal[2]);
        *s_c0 = c.pose ? c.Q[0] * sqrtf(d2g) + c.Q[1] * rot_angle(c, Re) + limit_penalty(c, q) +
                             (icol0 ? c.Q[2] : 0.f)
                       : c.Q[0] * d2g + limit_penalty(c, q);
      }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      const float oc = __shfl_xor(cl, d, kWave);
      const int oi = __shfl_xor(idx, d, kWave);
      if (oc < cl || (oc == cl && oi < idx)) {
        cl = oc;
        idx = oi;
      }
    }
    if (tid == 0) s_closest = n_obs > 0 ? idx : -1;
    // Broad phase (unicycle): every state of a rollout lies within
    // reach = max|v| N dt of p(x_t), so an obstacle whose surface is farther
    // than that (with a margin far above the FP32 rounding of the positions)
    // is never in contact; it is left out of the collision loops.  The kept
    // obstacles stay in index order, so the lowest-index rule is unchanged.
    // A moving obstacle covers at most |v| N dt more.
    bool keep = tid < n_obs;
    if (DYN == 0 && keep && c.reach < INFINITY) {
      const float R = c.robot_r + L.r[tid];
      const float d = sqrtf(dist2_2(x_t[0], x_t[1], L.o[tid].x, L.o[tid].y));
      const float4 v = L.v[tid];
      const float ov = sqrtf(v.x * v.x + v.y * v.y) * ((float)c.N * c.dt);
      const float ext = c.reach + R + ov;
      keep = !(d > ext + (1e-3f * ext + 1e-3f));
    }
    const unsigned long long m = __ballot(keep);
    if (keep) {
      const int pos = __popcll(m & ((1ull << tid) - 1ull));
      L.live[pos] = L.o[tid];
      L.vlive[pos] = L.v[tid];
      L.idx[pos] = tid;
    }
    if (tid == 0) L.n_live = __popcll(m);
  }
  __syncthreads();
}

// Block 0: push the observation into the history ring and publish the
// per-replan facts of the prologue.
__device__ void publish(const Cfg& c, const Bufs& b, const float* __restrict__ obs, int n_obs,
                        int bad, int closest, const float* p0, uint32_t step) {
  Ctrl* ct = b.ctrl;
  __shared__ int s_nh;
  if (threadIdx.x == 0) {
    int head = ct->hist_head;
    s_nh = (head + 1) % c.H;
  }
  __syncthreads();
  const int nh = s_nh;
  if (!bad) {
    for (int t = threadIdx.x; t < n_obs * c.p; t += kRollThreads) {
      const int i = t / c.p, d = t % c.p;
      b.hist[((size_t)nh * c.max_obs + i) * c.p + d] = obs[i * (c.p + 1) + d];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (!bad) {
      const int count = ct->hist_nobs == n_obs ? ct->hist_count : 0;
      ct->hist_head = nh;
      ct->hist_count = count + 1 < c.H ? count + 1 : c.H;
      ct->hist_nobs = n_obs;
    }
    ct->n_obs = n_obs;
    ct->nonfinite = bad;
    ct->closest = closest;
    ct->p0[0] = p0[0];
    ct->p0[1] = p0[1];
    ct->p0[2] = p0[2];
    ct->step_used = step;
  }
}

// Per-rollout contribution to the block partial record.
__device__ __forceinline__ void rollout_contrib(float* rec, bool active, int col, int first,
                                                int closest, float S, const float* src, int P) {
  // every field as one select, written as three 16-byte stores
  const bool hit = active && col;
  const bool inA = hit && first == closest;
  const bool feas = active && !col;
  float4* r4 = reinterpret_cast<float4*>(rec);
  static_assert(kPart == 12 && P_NCOL == 0 && P_NREF == 1 && P_NFEAS == 2 && P_SMIN_ALL == 3 &&
                    P_SMIN_FEAS == 4 && P_SUM_REF == 5 && P_SUM_COL == 8,
                "record layout");
  const float s0 = src[0], s1 = src[1], s2 = P == 3 ? src[2] : 0.f;
  r4[0] = make_float4(hit ? 1.f : 0.f, inA ? 1.f : 0.f, feas ? 1.f : 0.f, active ? S : INFINITY);
  r4[1] = make_float4(feas ? S : INFINITY, inA ? s0 : 0.f, inA ? s1 : 0.f, inA ? s2 : 0.f);
  r4[2] = make_float4(hit ? s0 : 0.f, hit ? s1 : 0.f, hit ? s2 : 0.f, 0.f);
}

// Partial records of groups of kGroup consecutive rollouts, each summed in
// rollout order: the grouping (and so every rounding) is the same however
// the rollouts were spread over waves, blocks or loop rounds.  recs holds the
// rpb records of the block's rollouts bx*rpb .. bx*rpb+rpb-1.
__device__ __forceinline__ void write_group_partials(const Bufs& b, float (*recs)[kPart], int rpb, int bx) {
  __syncthreads();
  const int ng = rpb / kGroup;
  for (int t = threadIdx.x; t < ng * kPart; t += kRollThreads) {
    const int g = t / kPart, f = t - g * kPart;
    const bool mn = f == P_SMIN_ALL || f == P_SMIN_FEAS;
    float acc = mn ? INFINITY : 0.f;
    for (int r = 0; r < kGroup; ++r) {
      const float v = recs[g * kGroup + r][f];
      acc = mn ? fminf(acc, v) : acc + v;
    }
    b.part[((size_t)bx * ng + g) * kPart + f] = acc;
  }
}

// Unicycle perturbation (Eq. (3)) of one control step: e = L g, the clamp to
// the bounds, and the applied perturbation (clamped control - nominal); all
// zero when `on` is false.
__device__ __forceinline__ void perturb_clamp(const Cfg& c, float n0, float n1, float g0, float g1, bool on,
                                              float& uv, float& uw, float& a0, float& a1) {
  const float e0 = c.L[0] * g0;
  const float e1 = c.L[2] * g0 + c.L[3] * g1;
  const float t0 = n0 + e0, t1 = n1 + e1;
  const float v = fminf(fmaxf(t0, c.umin[0]), c.umax[0]);
  const float w = fminf(fmaxf(t1, c.umin[1]), c.umax[1]);
  uv = on ? v : 0.f;
  uw = on ? w : 0.f;
  a0 = on ? (v == t0 ? e0 : v - n0) : 0.f;
  a1 = on ? (w == t1 ? e1 : w - n1) : 0.f;
}

// ---------------------------------------------------------------------------
// Unicycle rollouts (Sec. III-A): state (x, y, theta), control (v, omega).
// R rounds per wave: each wave runs R rollouts per block item, the nominal
// sequence staying in registers between rounds.  CVM as for the prologue.
template <int SEG, int R = 1, int CVM = 2>
__device__ __forceinline__ void rollout_unicycle_body(const Cfg& c, const Bufs& b, int bx, int by,
                                                      int nbx, const float* __restrict__ x_t,
                                                      const float* __restrict__ obs, int n_obs) {
  __shared__ ObsLds L;
  __shared__ int s_bad, s_closest;
  __shared__ float s_p0[3];
  __shared__ __align__(16) float s_rec[kRollWaves * (kWave / SEG) * R][kPart];
  // With one or two rounds the prologue (obstacles, finiteness, o*) runs
  // after the first round's noise, dynamics and cost, which do not need it,
  // so that its loads and barriers overlap that work; nothing is stored
  // before it has run.  With more rounds it runs first (the late form costs
  // registers, and so occupancy, in the persistent batched launch).
  constexpr bool LATE = R <= 2;
  const uint32_t step = b.ctrl->step_lo;
  int bad = 0, closest = -1;
  if constexpr (!LATE) {
    prologue<0, CVM>(c, b, x_t, obs, n_obs, L, s_bad, s_closest, s_p0);
    bad = s_bad;
    closest = s_closest;
    if (bx == 0) publish(c, b, obs, n_obs, bad, closest, s_p0, step);
  }
  const bool cv = CVM == 2 ? c.cv != 0 : CVM == 1;

  constexpr int SPW = kWave / SEG;
  constexpr int RPB = kRollWaves * SPW * R;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int j = lane & (SEG - 1), sgi = lane / SEG;
  const int N = c.N;
  const float dt = c.dt;
  const float x0 = x_t[0], y0 = x_t[1], th0 = x_t[2];
  const float n0 = j < N ? b.U[j * 2] : 0.f, n1 = j < N ? b.U[j * 2 + 1] : 0.f;
  // Paired rounds (R even): one Philox evaluation per lane serves two
  // rounds.  A rollout needs ceil(2N/4) counter blocks: at most 32 with
  // 64-lane segments, at most 16 with 32-lane ones (N <= 31), so the 64
  // lanes own, in groups of OWN, every block of the SPW rollouts of round
  // rr and of round rr + 1.  Each lane then takes the words of its own block
  // (j >> 1) from the owner lane, so every Gaussian is the one
  // step_gaussians<2> would give.
  constexpr bool PAIRED = R >= 2 && (R % 2) == 0;
  constexpr int OWN = SEG == 64 ? 32 : 16;
  // Rounds go RS at a time.  With paired Philox the two rounds that share an
  // evaluation also share one instruction stream up to the cost, so their
  // dependent chains (the DPP scans, the transcendentals) interleave; the
  // arithmetic of each rollout is unchanged.
  constexpr int RS = PAIRED ? 2 : 1;
  for (int r0 = 0; r0 < R; r0 += RS) {
  int kloc[RS], k[RS];
  bool inr[RS];
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    kloc[s] = ((r0 + s) * kRollWaves + wave) * SPW + sgi;
    // one rollout per wave with 64-lane segments: k is wave-uniform (scalar)
    k[s] = SEG == 64 ? __builtin_amdgcn_readfirstlane(bx * RPB + kloc[s]) : bx * RPB + kloc[s];
    inr[s] = k[s] < c.K;
  }

  // noise, perturbation and clamp (Eq. (3)); applied perturbation kept
  float uv[RS], uw[RS], a0[RS], a1[RS];
  if constexpr (PAIRED) {
    uint32_t pw[4] = {0u, 0u, 0u, 0u};
    {
      const int q = lane / OWN, ob = lane % OWN;
      const int orr = r0 + q / SPW, osg = q % SPW;
      const int ok = bx * RPB + (orr * kRollWaves + wave) * SPW + osg;
      if (ok < c.K && ob < c.B) philox((uint32_t)ob, (uint32_t)ok, step, c.stream_id, c.seed_lo, c.seed_hi, pw);
    }
#pragma unroll
    for (int s = 0; s < RS; ++s) {
      const int src = (s * SPW + sgi) * OWN + (j >> 1);
      uint32_t qw[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) qw[i] = (uint32_t)__shfl((int)pw[i], src, kWave);
      const bool odd = (j & 1) != 0;
      float g0, g1;
      box_muller(odd ? qw[2] : qw[0], odd ? qw[3] : qw[1], g0, g1);
      perturb_clamp(c, n0, n1, g0, g1, inr[s] && j < N, uv[s], uw[s], a0[s], a1[s]);
    }
  } else {
    uv[0] = uw[0] = a0[0] = a1[0] = 0.f;
    if (inr[0] && j < N) {
      float g[2];
      step_gaussians<2>(c, step, k[0], j, g);
      perturb_clamp(c, n0, n1, g[0], g[1], true, uv[0], uw[0], a0[0], a1[0]);
    }
  }
  // forward simulation, Eq. (4)/(21): heading and position are prefix sums
  float th[RS], sn[RS], cs[RS], px[RS], py[RS], S[RS];
#pragma unroll
  for (int s = 0; s < RS; ++s) th[s] = th0 + seg_excl_scan<SEG>(uw[s] * dt, j);
#pragma unroll
  for (int s = 0; s < RS; ++s) __sincosf(th[s], &sn[s], &cs[s]);
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    px[s] = x0 + seg_excl_scan<SEG>(uv[s] * cs[s] * dt, j);
    py[s] = y0 + seg_excl_scan<SEG>(uv[s] * sn[s] * dt, j);
  }
  // cost, Eq. (5): stage terms in lanes 0..N-1, terminal term in lane N
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const float lx = sq(px[s] - c.goal[0]), ly = sq(py[s] - c.goal[1]), lth = sq(th[s] - c.goal[2]);
    const float ls = c.Q[0] * lx + c.Q[1] * ly + c.Q[2] * lth + c.R[0] * uv[s] * uv[s] + c.R[1] * uw[s] * uw[s];
    const float lt = c.Qf[0] * lx + c.Qf[1] * ly + c.Qf[2] * lth;
    const float l = !inr[s] ? 0.f : (j < N ? ls : (j == N ? lt : 0.f));
    S[s] = seg_sum<SEG>(l);
  }

  if (LATE && r0 == 0) {
    prologue<0, CVM>(c, b, x_t, obs, n_obs, L, s_bad, s_closest, s_p0);
    bad = s_bad;
    closest = s_closest;
    if (bx == 0) publish(c, b, obs, n_obs, bad, closest, s_p0, step);
  }
#pragma unroll
  for (int s = 0; s < RS; ++s) {
  const bool act = inr[s] && !bad;
  if (act && j < N) {
    float2* ep = reinterpret_cast<float2*>(b.eps + ((size_t)k[s] * N + j) * 2);
    *ep = make_float2(a0[s], a1[s]);
  }

  // collision of states 1..N against the obstacles: lowest index hit
  // pass 1: does this state touch any obstacle?  pass 2 (only in waves with
  // a contact): the lowest obstacle index touched
  // (constant-velocity obstacles: obstacle i at o_i + j dt v_i for state j)
  const bool chk = act && j >= 1 && j <= N;
  const int n_live = L.n_live;
  const float tj = (float)j * dt;
  const float qx = px[s], qy = py[s];
  bool any = false;
  if (chk) {
    if (cv) {
      for (int i = 0; i < n_live; ++i) {
        const float4 o = L.live[i], v = L.vlive[i];
        any |= dist2_2(qx, qy, __builtin_fmaf(tj, v.x, o.x), __builtin_fmaf(tj, v.y, o.y)) <= o.w;
      }
    } else {
      for (int i = 0; i < n_live; ++i) {
        const float4 o = L.live[i];
        any |= dist2_2(qx, qy, o.x, o.y) <= o.w;
      }
    }
  }
  int hit = kInt32Max;
  if (__ballot(any) != 0ull && any) {
    if (cv) {
      for (int i = n_live - 1; i >= 0; --i) {
        const float4 o = L.live[i], v = L.vlive[i];
        hit = dist2_2(qx, qy, __builtin_fmaf(tj, v.x, o.x), __builtin_fmaf(tj, v.y, o.y)) <= o.w
                  ? L.idx[i] : hit;
      }
    } else {
      for (int i = n_live - 1; i >= 0; --i) {
        const float4 o = L.live[i];
        hit = dist2_2(qx, qy, o.x, o.y) <= o.w ? L.idx[i] : hit;
      }
    }
  }
  // first colliding state of each segment (lowest lane with a hit)
  const unsigned long long hm = __ballot(hit != kInt32Max);
  const unsigned long long m0 = SEG == 64 ? hm : (hm & 0xffffffffull);
  const unsigned long long m1 = SEG == 64 ? 0ull : (hm >> 32);
  const int f0 = m0 ? __ffsll((long long)m0) - 1 : 0;
  const int f1 = m1 ? __ffsll((long long)m1) - 1 : 0;
  const int col = (sgi == 0 ? m0 : m1) != 0ull;
  const int f = seg_pick_i<SEG>(hit, f0, f1);
  const float pfx = seg_pick<SEG>(qx, f0, f1), pfy = seg_pick<SEG>(qy, f0, f1);
  const int ln = N < SEG ? N : SEG - 1;
  const float ptx = seg_bcast<SEG>(qx, ln), pty = seg_bcast<SEG>(qy, ln);

  float src[2];
  src[0] = c.ref_mode == 1 ? pfx : ptx;
  src[1] = c.ref_mode == 1 ? pfy : pty;
  if (j == 0) {
    const int kk = k[s];
    if (act) {
      b.S[kk] = S[s];
      b.col[kk] = col;
      b.first[kk] = col ? f : -1;
      b.pT[2 * kk] = ptx;
      b.pT[2 * kk + 1] = pty;
      b.pF[2 * kk] = col ? pfx : 0.f;
      b.pF[2 * kk + 1] = col ? pfy : 0.f;
      // unit terminal displacement, Eq. (15)
      const float ex = ptx - x0, ey = pty - y0;
      const float den = __builtin_amdgcn_sqrtf(__builtin_fmaf(ey, ey, ex * ex)) + c.norm_eps;
      const float inv = __builtin_amdgcn_rcpf(den);  // v_sqrt_f32 and one v_rcp_f32
      b.g[2 * kk] = ex * inv;
      b.g[2 * kk + 1] = ey * inv;
    }
    rollout_contrib(s_rec[kloc[s]], act, col, col ? f : -1, closest, S[s], src, 2);
  }
  }
  }
  write_group_partials(b, s_rec, RPB, bx);
}

template <int SEG, int CV, int R>
__global__ __launch_bounds__(kRollThreads) void k_rollout_unicycle(Cfg c, Bufs b, const float* __restrict__ x_t, const float* __restrict__ obs, int n_obs) {
  rollout_unicycle_body<SEG, R, CV>(c, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, x_t, obs, n_obs);
}

// ---------------------------------------------------------------------------
// Six-joint arm rollouts (Sec. III-C): joint-velocity control, q_{j+1} =
// q_j + u_j dt; end-effector cost (squared distance, or the pose cost of the
// real-robot experiment), joint-limit penalty, link spheres against obstacle
// spheres.  Lane j of a segment holds control u_j and the state x_{j+1} it
// leads to (an inclusive scan), so N <= 32 fits a 32-lane segment and a wave
// runs two rollouts; the state part of the cost of x_t (the same for every
// rollout) comes from the prologue.
template <int SEG, int R = 1>
__device__ __forceinline__ void rollout_arm_body(const Cfg& c, const Bufs& b, int bx, int by, int nbx,
                                                 const float* __restrict__ x_t,
                                                 const float* __restrict__ obs, int n_obs) {
  constexpr int SPW = kWave / SEG;
  constexpr int RPB = kRollWaves * SPW * R;
  __shared__ ObsLds L;
  __shared__ int s_bad, s_closest;
  __shared__ float s_p0[3], s_c0;
  __shared__ __align__(16) float s_rec[RPB][kPart];
  prologue<1>(c, b, x_t, obs, n_obs, L, s_bad, s_closest, s_p0, &s_c0);
  const uint32_t step = b.ctrl->step_lo;
  const int bad = s_bad, closest = s_closest;
  if (bx == 0) publish(c, b, obs, n_obs, bad, closest, s_p0, step);
  const float c0 = s_c0;

  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const int j = lane & (SEG - 1), sgi = lane / SEG;
  const int N = c.N;
  const float dt = c.dt;
  float un[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) un[i] = j < N ? b.U[j * 6 + i] : 0.f;
  for (int rr = 0; rr < R; ++rr) {
  const int kloc = (rr * kRollWaves + wave) * SPW + sgi;
  const int k = SEG == 64 ? __builtin_amdgcn_readfirstlane(bx * RPB + kloc) : bx * RPB + kloc;
  const bool act = (k < c.K) && !bad;
  const bool live = act && j < N;  // control u_j, state x_{j+1}
  const bool last = j == N - 1;    // state x_N: terminal weights

  float u[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) u[i] = 0.f;
  if (live) {
    float g[6];
    step_gaussians<6>(c, step, k, j, g);
    float a[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      float e = 0.f;
#pragma unroll
      for (int cc = 0; cc < 6; ++cc)
        if (cc <= i) e += c.L[i * 6 + cc] * g[cc];
      const float n0 = un[i];
      const float t = n0 + e;
      u[i] = fminf(fmaxf(t, c.umin[i]), c.umax[i]);
      a[i] = u[i] == t ? e : u[i] - n0;
    }
    float2* ep = reinterpret_cast<float2*>(b.eps + ((size_t)k * N + j) * 6);
    ep[0] = make_float2(a[0], a[1]);
    ep[1] = make_float2(a[2], a[3]);
    ep[2] = make_float2(a[4], a[5]);
  }
  float q[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) q[i] = x_t[i] + seg_incl_scan<SEG>(u[i] * dt, j);
  float P[7][3], Re[9];
  arm_origins(c, q, P, Re);
  const float ex = P[6][0], ey = P[6][1], ez = P[6][2];
  float l = 0.f;
  const float d2g = sq(ex - c.goal[0]) + sq(ey - c.goal[1]) + sq(ez - c.goal[2]);
  if (live) {
    float r = 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) r += c.R[i] * u[i] * u[i];
    if (c.pose)  // Sec. III-C: w_p |p_ee - p_g| + w_R d_R (+ w_c I_col, below)
      l = (last ? c.Qf[0] : c.Q[0]) * sqrtf(d2g) + (last ? c.Qf[1] : c.Q[1]) * rot_angle(c, Re) +
          limit_penalty(c, q) + r;
    else
      l = (last ? c.Qf[0] : c.Q[0]) * d2g + limit_penalty(c, q) + r;
  }

  // pass 1: any contact of any link sphere with any obstacle (at time
  // (j + 1) dt for moving obstacles); pass 2 (waves with a contact): the
  // lowest obstacle index touched
  const float tj = (float)(j + 1) * dt;
  bool any = false;
  if (live) {
    for (int s = 0; s < c.ns; ++s) {
      float sx, sy, sz;
      sphere_centre(c, P, s, sx, sy, sz);
      if (c.cv) {
        for (int i = 0; i < n_obs; ++i) {
          const float4 o = L.o[i], v = L.v[i];
          any |= dist2_3(sx, sy, sz, __builtin_fmaf(tj, v.x, o.x), __builtin_fmaf(tj, v.y, o.y),
                         __builtin_fmaf(tj, v.z, o.z)) <= o.w;
        }
      } else {
        for (int i = 0; i < n_obs; ++i) {
          const float4 o = L.o[i];
          any |= dist2_3(sx, sy, sz, o.x, o.y, o.z) <= o.w;
        }
      }
    }
  }
  if (c.pose && any) l += last ? c.Qf[2] : c.Q[2];
  const float S = seg_sum<SEG>(l) + c0;
  int hit = kInt32Max;
  if (__ballot(any) != 0ull && any) {
    for (int s = 0; s < c.ns; ++s) {
      float sx, sy, sz;
      sphere_centre(c, P, s, sx, sy, sz);
      int hs = kInt32Max;
      if (c.cv) {
        for (int i = n_obs - 1; i >= 0; --i) {
          const float4 o = L.o[i], v = L.v[i];
          hs = dist2_3(sx, sy, sz, __builtin_fmaf(tj, v.x, o.x), __builtin_fmaf(tj, v.y, o.y),
                       __builtin_fmaf(tj, v.z, o.z)) <= o.w ? i : hs;
        }
      } else {
        for (int i = n_obs - 1; i >= 0; --i) {
          const float4 o = L.o[i];
          hs = dist2_3(sx, sy, sz, o.x, o.y, o.z) <= o.w ? i : hs;
        }
      }
      hit = hs < hit ? hs : hit;
    }
  }
  // first colliding state of each segment (lowest lane with a hit)
  const unsigned long long hm = __ballot(hit != kInt32Max);
  const unsigned long long m0 = SEG == 64 ? hm : (hm & 0xffffffffull);
  const unsigned long long m1 = SEG == 64 ? 0ull : (hm >> 32);
  const int f0 = m0 ? __ffsll((long long)m0) - 1 : 0;
  const int f1 = m1 ? __ffsll((long long)m1) - 1 : 0;
  const int col = (sgi == 0 ? m0 : m1) != 0ull;
  const int f = seg_pick_i<SEG>(hit, f0, f1);
  const float pfx = seg_pick<SEG>(ex, f0, f1), pfy = seg_pick<SEG>(ey, f0, f1),
              pfz = seg_pick<SEG>(ez, f0, f1);
  const int ln = N - 1;
  const float ptx = seg_bcast<SEG>(ex, ln), pty = seg_bcast<SEG>(ey, ln), ptz = seg_bcast<SEG>(ez, ln);

  float src[3];
  src[0] = c.ref_mode == 1 ? pfx : ptx;
  src[1] = c.ref_mode == 1 ? pfy : pty;
  src[2] = c.ref_mode == 1 ? pfz : ptz;
  if (j == 0) {
    if (act) {
      b.S[k] = S;
      b.col[k] = col;
      b.first[k] = col ? f : -1;
      b.pT[3 * k] = ptx;
      b.pT[3 * k + 1] = pty;
      b.pT[3 * k + 2] = ptz;
      b.pF[3 * k] = col ? pfx : 0.f;
      b.pF[3 * k + 1] = col ? pfy : 0.f;
      b.pF[3 * k + 2] = col ? pfz : 0.f;
      const float dx = ptx - s_p0[0], dy = pty - s_p0[1], dz = ptz - s_p0[2];
      const float den =
          __builtin_amdgcn_sqrtf(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx))) + c.norm_eps;
      const float inv = __builtin_amdgcn_rcpf(den);
      b.g[3 * k] = dx * inv;
      b.g[3 * k + 1] = dy * inv;
      b.g[3 * k + 2] = dz * inv;
    }
    rollout_contrib(s_rec[kloc], act, col, col ? f : -1, closest, S, src, 3);
  }
  }
  write_group_partials(b, s_rec, RPB, bx);
}

template <int SEG>
__global__ __launch_bounds__(kRollThreads) void k_rollout_arm(Cfg c, Bufs b, const float* __restrict__ x_t, const float* __restrict__ obs, int n_obs) {
  rollout_arm_body<SEG>(c, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, x_t, obs, n_obs);
}

// ---------------------------------------------------------------------------
// Batched rollouts: one persistent launch per rollout kind covers the rollout
// blocks of every planner of that kind in the batch; R rounds per wave.
template <int SEG, int R>
__global__ __launch_bounds__(kRollThreads) void kb_rollout_unicycle(CSlotStatic st, CSlotIO io, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kRollThreads>(t, s_pref, [&](int slot, int local) {
    const SlotStatic& S = *(const SlotStatic*)(st + slot);
    const SlotIO& I = *(const SlotIO*)(io + slot);
    rollout_unicycle_body<SEG, R>(S.c, S.b, local, 0, 0, I.x_t, I.obs, I.n_obs);
  });
}

template <int R>
__global__ __launch_bounds__(kRollThreads) void kb_rollout_arm(CSlotStatic st, CSlotIO io, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kRollThreads>(t, s_pref, [&](int slot, int local) {
    const SlotStatic& S = *(const SlotStatic*)(st + slot);
    const SlotIO& I = *(const SlotIO*)(io + slot);
    // the segment width is the member's own (a block-uniform branch)
    if (S.c.seg == 32)
      rollout_arm_body<32, R>(S.c, S.b, local, 0, 0, I.x_t, I.obs, I.n_obs);
    else
      rollout_arm_body<64, R>(S.c, S.b, local, 0, 0, I.x_t, I.obs, I.n_obs);
  });
}

// ---------------------------------------------------------------------------
// The same reduction on rollout records already in the planner buffers
// (records supplied by the caller): grid = nblk_roll blocks of rpb rollouts.
template <int DYN>
__global__ __launch_bounds__(kRollThreads) void k_reduce_records(Cfg c, Bufs b,
                                                                 const float* __restrict__ x_t,
                                                                 const float* __restrict__ obs,
                                                                 int n_obs) {
  __shared__ ObsLds L;
  __shared__ int s_bad, s_closest;
  __shared__ float s_p0[3];
  __shared__ __align__(16) float s_rec[kMaxRpb][kPart];
  prologue<DYN>(c, b, x_t, obs, n_obs, L, s_bad, s_closest, s_p0);
  const uint32_t step = b.ctrl->step_lo;
  const int bad = s_bad, closest = s_closest;
  if (blockIdx.x == 0) publish(c, b, obs, n_obs, bad, closest, s_p0, step);
  const int P = DYN == 0 ? 2 : 3;
  if (threadIdx.x < c.rpb) {
    const int k = blockIdx.x * c.rpb + threadIdx.x;
    const bool act = k < c.K && !bad;
    int col = 0, f = -1;
    float S = 0.f, src[3] = {0.f, 0.f, 0.f};
    if (act) {
      col = b.col[k];
      f = b.first[k];
      S = b.S[k];
      const float* sp = c.ref_mode == 1 ? b.pF : b.pT;
      for (int i = 0; i < P; ++i) src[i] = sp[(size_t)k * P + i];
      // Eq. (15) from the supplied terminal point
      float e[3] = {0.f, 0.f, 0.f};
      for (int i = 0; i < P; ++i) e[i] = b.pT[(size_t)k * P + i] - s_p0[i];
      const float den =
          sqrtf(__builtin_fmaf(e[2], e[2], __builtin_fmaf(e[1], e[1], e[0] * e[0]))) + c.norm_eps;
      const float inv = __builtin_amdgcn_rcpf(den);
      for (int i = 0; i < P; ++i) b.g[(size_t)k * P + i] = e[i] * inv;
    }
    rollout_contrib(s_rec[threadIdx.x], act, col, f, closest, S, src, P);
  }
  write_group_partials(b, s_rec, c.rpb, (int)blockIdx.x);
}

// Philox words and standard normals of every rollout (stage entry point):
// one thread per (rollout, counter block).
__global__ void k_stage_noise(Cfg c, uint32_t step, uint32_t* __restrict__ words,
                              float* __restrict__ gauss) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= c.K * c.B) return;
  const int k = t / c.B, bl = t % c.B;
  uint32_t w[4];
  philox((uint32_t)bl, (uint32_t)k, step, c.stream_id, c.seed_lo, c.seed_hi, w);
  if (words) {
    uint4* wp = reinterpret_cast<uint4*>(words) + t;
    *wp = make_uint4(w[0], w[1], w[2], w[3]);
  }
  if (gauss) {
    for (int h = 0; h < 2; ++h) {
      const int e = 4 * bl + 2 * h;
      if (e >= c.NM) break;
      float ga, gb;
      box_muller(w[2 * h], w[2 * h + 1], ga, gb);
      gauss[(size_t)k * c.NM + e] = ga;
      if (e + 1 < c.NM) gauss[(size_t)k * c.NM + e + 1] = gb;
    }
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// kind 0: unicycle on 32-lane segments, 1: unicycle on 64 lanes, 2: arm;
// r: rounds per wave (1, 2, 4 or 8)
template <int R>
static void launch_batch_rollout_r(Launcher& L, int kind, CSlotStatic st, CSlotIO io, Tab t, int grid) {
  if (kind == 0) L(kb_rollout_unicycle<32, R>, dim3(grid), dim3(kRollThreads), st, io, t);
  else if (kind == 1) L(kb_rollout_unicycle<64, R>, dim3(grid), dim3(kRollThreads), st, io, t);
  else L(kb_rollout_arm<R>, dim3(grid), dim3(kRollThreads), st, io, t);
}

void launch_batch_rollout(Launcher& L, int kind, int r, const SlotStatic* st, const SlotIO* io, Tab t,
                          int grid) {
  if (grid <= 0) return;
  const CSlotStatic cst = (CSlotStatic)st;
  const CSlotIO cio = (CSlotIO)io;
  switch (r) {
    case 2: launch_batch_rollout_r<2>(L, kind, cst, cio, t, grid); break;
    case 4: launch_batch_rollout_r<4>(L, kind, cst, cio, t, grid); break;
    case 8: launch_batch_rollout_r<8>(L, kind, cst, cio, t, grid); break;
    default: launch_batch_rollout_r<1>(L, kind, cst, cio, t, grid); break;
  }
}

void launch_rollout(Launcher& L, const Cfg& c, const Bufs& b, const float* x_t, const float* obs,
                    int n_obs) {
  dim3 grid(c.nblk_roll), block(kRollThreads);
  if (c.dyn == 0) {
    // R rounds per wave: the block count shrinks by R; the partial records
    // (fixed groups of kGroup rollouts) do not depend on it
    using KFn = void (*)(Cfg, Bufs, const float*, const float*, int);
    KFn f;
    if (c.seg == 32)
      f = c.roll_r == 2 ? (c.cv ? k_rollout_unicycle<32, 1, 2> : k_rollout_unicycle<32, 0, 2>)
                        : (c.cv ? k_rollout_unicycle<32, 1, 1> : k_rollout_unicycle<32, 0, 1>);
    else
      f = c.roll_r == 2 ? (c.cv ? k_rollout_unicycle<64, 1, 2> : k_rollout_unicycle<64, 0, 2>)
                        : (c.cv ? k_rollout_unicycle<64, 1, 1> : k_rollout_unicycle<64, 0, 1>);
    const int rr = c.roll_r == 2 ? 2 : 1;
    L(f, dim3((c.K + c.rpb * rr - 1) / (c.rpb * rr)), block, c, b, x_t, obs, n_obs);
  } else {
    L(c.seg == 32 ? k_rollout_arm<32> : k_rollout_arm<64>, grid, block, c, b, x_t, obs, n_obs);
  }
}

void launch_reduce_records(Launcher& L, const Cfg& c, const Bufs& b, const float* x_t,
                           const float* obs, int n_obs) {
  dim3 grid(c.nblk_roll), block(kRollThreads);
  if (c.dyn == 0)
    L(k_reduce_records<0>, grid, block, c, b, x_t, obs, n_obs);
  else
    L(k_reduce_records<1>, grid, block, c, b, x_t, obs, n_obs);
}

void launch_stage_noise(Launcher& L, const Cfg& c, uint32_t step, uint32_t* words, float* gauss) {
  const int total = c.K * c.B;
  L(k_stage_noise, dim3((total + 255) / 256), dim3(256), c, step, words, gauss);
}

}  // namespace cemppi
