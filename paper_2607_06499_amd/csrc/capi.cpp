// capi.cpp -- the C ABI of libcemppi.so (declared in include/cemppi.h):
// validation, the per-planner device arena and the launch sequence of one
// replan.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cemppi.h"
#include "device.hpp"
#include "launch.hpp"
#include "planner.hpp"

namespace cemppi {
void launch_rollout(Launcher& L, const Cfg& c, const Bufs& b, const float* x_t, const float* obs,
                    int n_obs);
void launch_reduce_records(Launcher& L, const Cfg& c, const Bufs& b, const float* x_t,
                           const float* obs, int n_obs);
void launch_stage_noise(Launcher& L, const Cfg& c, uint32_t step, uint32_t* words, float* gauss);
void launch_post_rollout(Launcher& L, const Cfg& c, const Bufs& b);
void launch_finish(Launcher& L, const Cfg& c, const Bufs& b, float* u_out, float* U_out, void* info);
void launch_stage_dbscan(Launcher& L, const Cfg& c, const Bufs& b, const float* z, int V,
                         int* ncount, int* label, int* mout);
}  // namespace cemppi

using namespace cemppi;

static_assert(sizeof(ce_mppi_info) == 4 * (12 + 2 + 10), "ce_mppi_info layout");

namespace {

thread_local std::string g_err;

ce_status fail(ce_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

ce_status hip_fail(hipError_t e, const char* what) {
  return fail(CE_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite(float x) { return std::isfinite(x); }

// Arena carving: every buffer 256-byte aligned.
struct Carver {
  size_t off = 0;
  template <class T>
  size_t take(size_t count) {
    const size_t o = off;
    off += ((count * sizeof(T) + 255) / 256) * 256;
    return o;
  }
};

void dims(int dyn, int& n, int& m, int& p) {
  if (dyn == CE_DYN_UNICYCLE) {
    n = 3; m = 2; p = 2;
  } else {
    n = 12; m = 6; p = 3;
  }
}

ce_status validate(const ce_mppi_config* c) {
  if (!c) return fail(CE_EINVAL, "config is NULL");
  if (c->abi_version != CE_MPPI_ABI_VERSION) return fail(CE_EINVAL, "abi_version mismatch");
  if (c->dynamics != CE_DYN_UNICYCLE && c->dynamics != CE_DYN_ARM6)
    return fail(CE_EINVAL, "unknown dynamics");
  if (c->horizon < 1 || c->horizon > CE_MPPI_MAX_HORIZON)
    return fail(CE_EINVAL, "horizon out of range 1..63");
  if (c->num_samples < 1 || c->num_samples > CE_MPPI_MAX_SAMPLES)
    return fail(CE_EINVAL, "num_samples out of range 1..65536");
  if (!(c->dt > 0.f) || !finite(c->dt)) return fail(CE_EINVAL, "dt must be finite and > 0");
  if (!(c->lambda > 0.f) || !finite(c->lambda)) return fail(CE_EINVAL, "lambda must be finite and > 0");
  if (!(c->dbscan_eps > 0.f) || !finite(c->dbscan_eps)) return fail(CE_EINVAL, "dbscan_eps must be > 0");
  if (c->dbscan_min_pts < 1) return fail(CE_EINVAL, "dbscan_min_pts must be >= 1");
  if (!(c->norm_eps >= 0.f) || !finite(c->norm_eps)) return fail(CE_EINVAL, "norm_eps must be >= 0");
  if (c->scene_mode != CE_SCENE_STATIC && c->scene_mode != CE_SCENE_DYNAMIC)
    return fail(CE_EINVAL, "unknown scene_mode");
  if (c->history_len < 1 || c->history_len > CE_MPPI_MAX_HISTORY)
    return fail(CE_EINVAL, "history_len out of range 1..16");
  if (c->scene_mode == CE_SCENE_DYNAMIC && c->history_len < 2)
    return fail(CE_EINVAL, "dynamic scenes need history_len >= 2");
  if (!(c->v_obs_min >= 0.f)) return fail(CE_EINVAL, "v_obs_min must be >= 0");
  if (c->ref_mode != CE_REF_TERMINAL && c->ref_mode != CE_REF_FIRST_CONTACT)
    return fail(CE_EINVAL, "unknown ref_mode");
  if (c->max_obstacles < 0 || c->max_obstacles > CE_MPPI_MAX_OBSTACLES)
    return fail(CE_EINVAL, "max_obstacles out of range 0..64");
  if (!(c->robot_radius >= 0.f) || !finite(c->robot_radius))
    return fail(CE_EINVAL, "robot_radius must be finite and >= 0");
  int n, m, p;
  dims(c->dynamics, n, m, p);
  for (int i = 0; i < 36; ++i)
    if (!finite(c->noise_chol[i])) return fail(CE_EINVAL, "noise_chol must be finite");
  for (int i = 0; i < m; ++i) {
    if (std::isnan(c->u_min[i]) || std::isnan(c->u_max[i]) || c->u_min[i] > c->u_max[i])
      return fail(CE_EINVAL, "control bounds must satisfy u_min <= u_max");
    if (!finite(c->goal[i]) || !finite(c->Q[i]) || !finite(c->R[i]) || !finite(c->Qf[i]))
      return fail(CE_EINVAL, "cost parameters must be finite");
  }
  if (c->flags & ~(CE_FLAG_POSE_COST | CE_FLAG_OBS_CONST_VEL))
    return fail(CE_EINVAL, "unknown flags");
  if ((c->flags & CE_FLAG_POSE_COST) && c->dynamics != CE_DYN_ARM6)
    return fail(CE_EINVAL, "the pose cost needs the arm dynamics");
  if ((c->flags & CE_FLAG_OBS_CONST_VEL) && c->history_len < 2)
    return fail(CE_EINVAL, "constant-velocity obstacles need history_len >= 2");
  if (c->dynamics == CE_DYN_ARM6) {
    if (c->n_link_spheres < 1 || c->n_link_spheres > CE_MPPI_MAX_SPHERES)
      return fail(CE_EINVAL, "n_link_spheres out of range 1..16");
    if (!(c->link_sphere_radius >= 0.f) || !finite(c->link_sphere_radius))
      return fail(CE_EINVAL, "link_sphere_radius must be finite and >= 0");
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 4; ++j)
        if (!finite(c->dh[i][j])) return fail(CE_EINVAL, "dh must be finite");
    double total = 0.0;
    for (int i = 0; i < 6; ++i) total += std::hypot((double)c->dh[i][0], (double)c->dh[i][1]);
    if (!(total > 0.0)) return fail(CE_EINVAL, "arm has zero length");
  }
  return CE_OK;
}

// Angular windows of the 2-D DBSCAN (cluster.hip, k_wdbscan), in
// double precision.  Ring points have |z| in [s_lo, s_hi]: the features of
// Eq. (13) are unit directions scaled by |d| / (|d| + eps_n), so this holds
// for every feasible rollout whose terminal point is more than about 1 mm
// from the reference point (others are tested against every point).  For a
// pair of ring points at angular separation phi,
//   4 s_lo^2 sin^2(phi/2) <= |a - b|^2 <= (s_hi - s_lo)^2 + 4 s_hi^2 sin^2(phi/2):
// below the inner angle the pair is surely within eps (FP32 rounding of the
// distance test is far inside the 1e-4 relative margin), above the outer
// angle surely not.  The windows lose the error of two computed angles
// (atan2f, the shift by pi and the scaling to buckets: well under 1e-5 rad
// each) and 1e-2 bucket for the rounding of u +- w.  Leaves w_g = 0 (path
// off) where the windows do not fit: 3-D features, an inner window under
// five buckets (eps below about 0.01) or an outer window of a quarter turn
// or more (eps above about 1.4).
void set_windows(Cfg& c) {
  const double pi = 3.14159265358979323846, beta = 2.0 * pi / kWinBins;
  const double delta = 1e-3;
  const double s_lo = (1.0 - delta) * (1.0 - 1e-6), s_hi = (1.0 + 2e-6) * (1.0 + 1e-6);
  const double e2 = (double)c.eps2;
  const double e_ang = 2e-5;
  c.w_scale = (float)(kWinBins / (2.0 * pi));
  c.w_r2lo = (float)((1.0 - delta) * (1.0 - delta));
  c.w_r2hi = (float)((1.0 + 2e-6) * (1.0 + 2e-6));
  c.w_in = c.w_out = 0.f;
  c.w_g = c.w_gout = 0;
  const double ain = (e2 * (1.0 - 1e-4) - (s_hi - s_lo) * (s_hi - s_lo)) / (4.0 * s_hi * s_hi);
  const double aout = e2 * (1.0 + 1e-4) / (4.0 * s_lo * s_lo);
  if (c.p != 2 || c.K > kWinMaxK || !(ain > 0.0) || !(aout < 0.5)) return;
  const double din = 2.0 * std::asin(std::sqrt(ain)), dout = 2.0 * std::asin(std::sqrt(aout));
  const double win = (din - e_ang) / beta - 1e-2, wout = (dout + e_ang) / beta + 1e-2;
  const int g = (int)std::floor(win) - 1, gout = (int)std::floor(wout) + 1;
  // runs need gaps of at least four buckets (at most kWinMaxRuns runs), and
  // only adjacent runs may be linked
  if (g < 3 || 2 * g + 2 <= gout) return;
  c.w_in = (float)win;
  c.w_out = (float)wout;
  c.w_g = g;
  c.w_gout = gout;
}

void build_cfg(const ce_mppi_config* u, Cfg& c) {
  std::memset(&c, 0, sizeof(c));
  c.dyn = u->dynamics;
  dims(c.dyn, c.n, c.m, c.p);
  c.N = u->horizon;
  c.K = u->num_samples;
  c.NM = c.N * c.m;
  c.B = (c.NM + 3) / 4;
  // lanes per rollout: the unicycle keeps x_0..x_N in lanes 0..N, the arm
  // keeps u_j and x_{j+1} in lane j
  c.seg = (c.dyn == CE_DYN_UNICYCLE ? c.N + 1 <= 32 : c.N <= 32) ? 32 : 64;
  c.rpb = kRollWaves * (64 / c.seg);
  c.nblk_roll = (c.K + c.rpb - 1) / c.rpb;
  c.roll_r = 1;
  // every rollout state lies within max|v| N dt of the start position (the
  // clamped speed bounds each step's displacement)
  {
    const double vmax = std::max(std::fabs((double)u->u_min[0]), std::fabs((double)u->u_max[0]));
    c.reach = (u->dynamics == CE_DYN_UNICYCLE && std::isfinite(vmax))
                  ? (float)(vmax * u->horizon * (double)u->dt)
                  : INFINITY;
  }
  c.npart = (c.K + kGroup - 1) / kGroup;
  c.dt = u->dt;
  c.lambda = u->lambda;
  c.norm_eps = u->norm_eps;
  for (int i = 0; i < 36; ++i) c.L[i] = u->noise_chol[i];
  for (int i = 0; i < 6; ++i) {
    c.umin[i] = u->u_min[i];
    c.umax[i] = u->u_max[i];
    c.goal[i] = u->goal[i];
    c.Q[i] = u->Q[i];
    c.R[i] = u->R[i];
    c.Qf[i] = u->Qf[i];
    c.qlim[i] = u->q_limit[i];
  }
  const float e = u->dbscan_eps;
  c.eps2 = e * e;
  c.min_pts = u->dbscan_min_pts;
  c.scene_mode = u->scene_mode;
  c.H = u->history_len;
  c.v_obs_min = u->v_obs_min;
  c.ref_mode = u->ref_mode;
  c.max_obs = u->max_obstacles;
  c.robot_r = u->robot_radius;
  c.wlim = u->w_limit;
  c.cv = (u->flags & CE_FLAG_OBS_CONST_VEL) ? 1 : 0;
  c.pose = (u->flags & CE_FLAG_POSE_COST) ? 1 : 0;
  {
    // goal orientation of the pose cost from its rotation vector (Rodrigues)
    const double r0 = u->goal[3], r1 = u->goal[4], r2 = u->goal[5];
    const double th = std::sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (c.pose && th > 0.0) {
      const double k0 = r0 / th, k1 = r1 / th, k2 = r2 / th;
      const double s = std::sin(th), v = 1.0 - std::cos(th);
      const double K[9] = {0, -k2, k1, k2, 0, -k0, -k1, k0, 0};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double kk = 0.0;
          for (int l = 0; l < 3; ++l) kk += K[i * 3 + l] * K[l * 3 + j];
          R[i * 3 + j] = (i == j ? 1.0 : 0.0) + s * K[i * 3 + j] + v * kk;
        }
    }
    for (int i = 0; i < 9; ++i) c.Rg[i] = (float)R[i];
  }
  if (c.dyn == CE_DYN_ARM6) {
    double seg[6], total = 0.0;
    for (int i = 0; i < 6; ++i) {
      const double a = u->dh[i][0], d = u->dh[i][1], al = u->dh[i][2];
      c.dh_a[i] = u->dh[i][0];
      c.dh_d[i] = u->dh[i][1];
      c.dh_ca[i] = (float)std::cos(al);
      c.dh_sa[i] = (float)std::sin(al);
      c.dh_off[i] = u->dh[i][3];
      seg[i] = std::sqrt(a * a + d * d);
      total += seg[i];
    }
    c.ns = u->n_link_spheres;
    c.rs = u->link_sphere_radius;
    // sphere s sits at arc length (s + 1/2)/ns of the frame-origin polyline;
    // segment lengths sqrt(a^2 + d^2) do not depend on the joint angles
    for (int s = 0; s < c.ns; ++s) {
      const double target = ((double)s + 0.5) / (double)c.ns * total;
      int i = 0;
      double start = 0.0;
      while (i < 5 && start + seg[i] < target) {
        start += seg[i];
        ++i;
      }
      c.sph_seg[s] = i;
      c.sph_t[s] = seg[i] > 0.0 ? (float)((target - start) / seg[i]) : 0.f;
    }
  }
  c.seed_lo = (uint32_t)(u->seed & 0xffffffffu);
  c.seed_hi = (uint32_t)(u->seed >> 32);
  c.stream_id = u->stream_id;
  c.ntile = (c.K + kTile - 1) / kTile;
  c.nblk_upd = (c.K + kUpdChunk - 1) / kUpdChunk;
  c.mcap = c.K;
  set_windows(c);
  c.dbpath = c.w_g > 0 ? 0 : (c.K <= kAdjMaxK ? 1 : 2);
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

namespace cemppi {
ce_status set_error(ce_status s, const std::string& msg) { return fail(s, msg); }
ce_status set_hip_error(hipError_t e, const char* what) { return hip_fail(e, what); }
}  // namespace cemppi

extern "C" {

ce_status ce_mppi_config_init(ce_mppi_config* cfg, int32_t dynamics) {
  if (!cfg) return fail(CE_EINVAL, "config is NULL");
  if (dynamics != CE_DYN_UNICYCLE && dynamics != CE_DYN_ARM6) return fail(CE_EINVAL, "unknown dynamics");
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->abi_version = CE_MPPI_ABI_VERSION;
  cfg->dynamics = dynamics;
  cfg->horizon = 30;
  cfg->num_samples = 1024;
  cfg->dt = 0.1f;
  cfg->lambda = 1.0f;
  int n, m, p;
  dims(dynamics, n, m, p);
  for (int i = 0; i < m; ++i) cfg->noise_chol[i * m + i] = 0.5f;
  for (int i = 0; i < 6; ++i) {
    cfg->u_min[i] = -INFINITY;
    cfg->u_max[i] = INFINITY;
    cfg->q_limit[i] = 3.14159265f;
  }
  cfg->dbscan_eps = 0.3f;
  cfg->dbscan_min_pts = 10;
  cfg->norm_eps = 1e-6f;
  cfg->scene_mode = CE_SCENE_STATIC;
  cfg->history_len = 5;
  cfg->v_obs_min = 1e-3f;
  cfg->ref_mode = CE_REF_TERMINAL;
  cfg->max_obstacles = CE_MPPI_MAX_OBSTACLES;
  cfg->n_link_spheres = 8;
  cfg->link_sphere_radius = 0.05f;
  cfg->w_limit = 100.0f;
  cfg->seed = 1;
  return CE_OK;
}

ce_status ce_mppi_create(const ce_mppi_config* cfg, ce_mppi_planner** out) {
  if (!out) return fail(CE_EINVAL, "out is NULL");
  *out = nullptr;
  ce_status st = validate(cfg);
  if (st != CE_OK) return st;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0) return fail(CE_EDEVICE, "no HIP device available");
  if (cfg->device < 0 || cfg->device >= ndev) return fail(CE_EINVAL, "device ordinal out of range");
  DeviceGuard guard(cfg->device);

  ce_mppi_planner* P = new (std::nothrow) ce_mppi_planner();
  if (!P) return fail(CE_ENOMEM, "host allocation failed");
  P->cfg = *cfg;
  build_cfg(cfg, P->c);
  {
    // Two rollout rounds per wave halve the per-block prologue when the
    // unicycle launch still has at least two blocks per compute unit; a
    // smaller grid (or the arm, whose waves are long) runs one round.
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess ||
        cus < 1)
      cus = 256;
    Cfg& cm = P->c;
    const int blocks2 = (cm.K + 2 * cm.rpb - 1) / (2 * cm.rpb);
    cm.roll_r = (cm.dyn == CE_DYN_UNICYCLE && blocks2 >= 2 * cus) ? 2 : 1;
  }
  const Cfg& c = P->c;
  const size_t K = (size_t)c.K, NM = (size_t)c.NM, p = (size_t)c.p;
  const size_t zs = c.p == 2 ? 2 : 4;
  const size_t nw = (K + 63) / 64 + 1;
  const size_t hist = (size_t)c.H * (size_t)(c.max_obs > 0 ? c.max_obs : 1) * p;
  Carver cv;
  const size_t o_ctrl = cv.take<Ctrl>(1);
  const size_t o_U = cv.take<float>(NM), o_Unew = cv.take<float>(NM), o_hist = cv.take<float>(hist);
  const size_t o_S = cv.take<float>(K), o_col = cv.take<int>(K), o_first = cv.take<int>(K);
  const size_t o_pT = cv.take<float>(K * p), o_pF = cv.take<float>(K * p), o_g = cv.take<float>(K * p);
  // (plus the chunks of the last row that the update kernel reads past its end)
  const size_t o_eps = cv.take<float>(K * NM + (size_t)kFinChunks * kWave);
  // room for the groups of the widest block (kMaxR rounds of 2 rollouts per wave)
  const size_t o_part = cv.take<float>((size_t)(c.npart + kMaxRpb * kMaxR / kGroup) * kPart);
  const size_t o_vidx = cv.take<int>(K), o_z = cv.take<float>(K * zs), o_gv = cv.take<float>(K * zs);
  const size_t o_Sv = cv.take<float>(K);
  const size_t o_zs = cv.take<float>(K * zs), o_sid = cv.take<int>(K);
  const size_t o_tlo = cv.take<float4>((size_t)c.ntile), o_thi = cv.take<float4>((size_t)c.ntile);
  const size_t o_nc = cv.take<int>(K), o_mcn = cv.take<int>(K), o_root = cv.take<int>(K);
  const size_t o_lab = cv.take<int>(K);
  const size_t o_cm = cv.take<unsigned long long>(nw), o_hm = cv.take<unsigned long long>(nw);
  const size_t o_tadj = cv.take<unsigned long long>(kMaxTrees);
  const bool with_adj = c.K <= kAdjMaxK;
  const size_t o_adj = cv.take<uint4>(with_adj ? (size_t)c.ntile * c.ntile * kTile : 0);
  const bool with_win = c.w_g > 0;
  const size_t wk = with_win ? K : 0;
  const size_t o_wcnt = cv.take<int>(with_win ? kWinBins + 1 : 0);
  const size_t o_wstart = cv.take<int>(with_win ? kWinBins + 2 : 0);
  const size_t o_wbmin = cv.take<int>(with_win ? kWinBins : 0);
  const size_t o_wkey = cv.take<int>(wk), o_wnc = cv.take<int>(wk);
  const size_t o_wuf = cv.take<int>(with_win ? 3 * (kWinMaxRuns + K) : 0);
  // (one region of K indices per block of the count pass, 512 positions each)
  const size_t o_wzone = cv.take<int>(with_win ? (K + kWinPos - 1) / kWinPos * K : 0);
  const size_t o_ccost = cv.take<float>((size_t)c.mcap), o_cdir = cv.take<float>((size_t)c.mcap * 4);
  const size_t o_csize = cv.take<int>((size_t)c.mcap), o_csmin = cv.take<float>((size_t)c.mcap);
  // update partials, then rows that stay zero so the final combination can
  // request whole batches of rows (kFinRows per wave) without bounds tests,
  // and the chunks of the last row that reach past its end
  const size_t o_upart = cv.take<float>((size_t)(c.nblk_upd + (kFinThreads / kWave) * kFinRows) * (NM + 1) +
                                        (size_t)kFinChunks * kWave);
  P->arena_bytes = cv.off;
  e = hipMalloc(&P->arena, P->arena_bytes);
  if (e != hipSuccess) {
    delete P;
    return fail(CE_ENOMEM, std::string("hipMalloc of the planner arena failed: ") + hipGetErrorString(e));
  }
  char* base = static_cast<char*>(P->arena);
  Bufs& b = P->b;
  b.ctrl = reinterpret_cast<Ctrl*>(base + o_ctrl);
  b.U = reinterpret_cast<float*>(base + o_U);
  b.Unew = reinterpret_cast<float*>(base + o_Unew);
  b.hist = reinterpret_cast<float*>(base + o_hist);
  b.S = reinterpret_cast<float*>(base + o_S);
  b.col = reinterpret_cast<int*>(base + o_col);
  b.first = reinterpret_cast<int*>(base + o_first);
  b.pT = reinterpret_cast<float*>(base + o_pT);
  b.pF = reinterpret_cast<float*>(base + o_pF);
  b.g = reinterpret_cast<float*>(base + o_g);
  b.eps = reinterpret_cast<float*>(base + o_eps);
  b.part = reinterpret_cast<float*>(base + o_part);
  b.vidx = reinterpret_cast<int*>(base + o_vidx);
  b.z = reinterpret_cast<float*>(base + o_z);
  b.gv = reinterpret_cast<float*>(base + o_gv);
  b.Sv = reinterpret_cast<float*>(base + o_Sv);
  b.zs = reinterpret_cast<float*>(base + o_zs);
  b.sid = reinterpret_cast<int*>(base + o_sid);
  b.tlo = reinterpret_cast<float4*>(base + o_tlo);
  b.thi = reinterpret_cast<float4*>(base + o_thi);
  b.ncount = reinterpret_cast<int*>(base + o_nc);
  b.mcn = reinterpret_cast<int*>(base + o_mcn);
  b.root = reinterpret_cast<int*>(base + o_root);
  b.label = reinterpret_cast<int*>(base + o_lab);
  b.coremask = reinterpret_cast<unsigned long long*>(base + o_cm);
  b.hookmask = reinterpret_cast<unsigned long long*>(base + o_hm);
  b.tadj = reinterpret_cast<unsigned long long*>(base + o_tadj);
  b.adj = with_adj ? reinterpret_cast<uint4*>(base + o_adj) : nullptr;
  b.wcnt = with_win ? reinterpret_cast<int*>(base + o_wcnt) : nullptr;
  b.wstart = with_win ? reinterpret_cast<int*>(base + o_wstart) : nullptr;
  b.wbmin = with_win ? reinterpret_cast<int*>(base + o_wbmin) : nullptr;
  b.wkey = with_win ? reinterpret_cast<int*>(base + o_wkey) : nullptr;
  b.wnc = with_win ? reinterpret_cast<int*>(base + o_wnc) : nullptr;
  b.wuf = with_win ? reinterpret_cast<int*>(base + o_wuf) : nullptr;
  b.wzone = with_win ? reinterpret_cast<int*>(base + o_wzone) : nullptr;
  b.c_cost = reinterpret_cast<float*>(base + o_ccost);
  b.c_dir = reinterpret_cast<float*>(base + o_cdir);
  b.c_size = reinterpret_cast<int*>(base + o_csize);
  b.c_smin = reinterpret_cast<float*>(base + o_csmin);
  b.upart = reinterpret_cast<float*>(base + o_upart);
  e = hipMemset(P->arena, 0, P->arena_bytes);
  if (e == hipSuccess) {
    Ctrl init;
    std::memset(&init, 0, sizeof(init));
    init.hist_head = c.H - 1;
    init.hist_nobs = -1;
    init.hs_head = c.H - 1;
    init.hs_nobs = -1;
    e = hipMemcpy(b.ctrl, &init, sizeof(init), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(P->arena);
    delete P;
    return hip_fail(e, "planner initialisation");
  }
  P->cap_K = K;
  *out = P;
  return CE_OK;
}

namespace {
void drop_graph(ReplanGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = ReplanGraph();
}

void drop_timing(Timing& t) {
  for (hipEvent_t e : t.ev) (void)hipEventDestroy(e);
  t = Timing();
}

hipError_t build_graph(ce_mppi_planner* P, const float* x_t, const float* obs, int n_obs, float* u_out,
                       float* U_out, void* info) {
  ReplanGraph& g = P->g;
  hipError_t e = hipGraphCreate(&g.graph, 0);
  if (e != hipSuccess) return e;
  Launcher L(nullptr, g.graph);
  launch_rollout(L, P->c, P->b, x_t, obs, n_obs);
  launch_post_rollout(L, P->c, P->b);
  launch_finish(L, P->c, P->b, u_out, U_out, info);
  if (L.err != hipSuccess) return L.err;
  g.first = L.nodes.front();
  g.last = L.nodes.back();
  e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return e;
  g.x = x_t;
  g.obs = obs;
  g.n_obs = n_obs;
  g.u_out = u_out;
  g.U_out = U_out;
  g.info = info;
  return hipSuccess;
}

hipError_t replan_graph(ce_mppi_planner* P, const float* x_t, const float* obs, int n_obs,
                        float* u_out, float* U_out, void* info, hipStream_t s) {
  ReplanGraph& g = P->g;
  hipError_t e = hipSuccess;
  if (!g.exec) {
    e = build_graph(P, x_t, obs, n_obs, u_out, U_out, info);
    if (e != hipSuccess) {
      drop_graph(g);
      return e;
    }
  }
  if (x_t != g.x || obs != g.obs || n_obs != g.n_obs) {
    Cfg c = P->c;
    Bufs b = P->b;
    const float* xx = x_t;
    const float* oo = obs;
    int nn = n_obs;
    e = set_node_args(g.exec, g.first, c, b, xx, oo, nn);
    if (e != hipSuccess) return e;
    g.x = x_t;
    g.obs = obs;
    g.n_obs = n_obs;
  }
  if (u_out != g.u_out || U_out != g.U_out || info != g.info) {
    Cfg c = P->c;
    Bufs b = P->b;
    float* uo = u_out;
    float* Uo = U_out;
    void* in = info;
    e = set_node_args(g.exec, g.last, c, b, uo, Uo, in);
    if (e != hipSuccess) return e;
    g.u_out = u_out;
    g.U_out = U_out;
    g.info = info;
  }
  return hipGraphLaunch(g.exec, s);
}
}  // namespace

void ce_mppi_destroy(ce_mppi_planner* P) {
  if (!P) return;
  {
    DeviceGuard guard(P->cfg.device);
    drop_graph(P->g);
    drop_timing(P->t);
    if (P->arena) (void)hipFree(P->arena);
  }
  delete P;
}

}  // extern "C"

namespace {
// A replan on a stream other than the previous replan's while that stream
// still has work queued: the previous replan may still be running.
ce_status check_not_busy(ce_mppi_planner* P, hipStream_t s) {
  if (!P->used || s == P->last_stream) return CE_OK;
  const hipError_t q = hipStreamQuery(P->last_stream);
  if (q == hipSuccess) return CE_OK;
  if (q == hipErrorNotReady)
    return fail(CE_EBUSY, "the planner's previous replan may still be in flight on another stream");
  return hip_fail(q, "hipStreamQuery");
}
}  // namespace

namespace cemppi {
void mark_stream(ce_mppi_planner* P, hipStream_t s) {
  P->last_stream = s;
  P->used = true;
}
}  // namespace cemppi

namespace cemppi {
ce_status replan_unchecked(ce_mppi_planner* P, const float* x_t, const float* obstacles,
                                   int32_t n_obs, float* u_out, float* U_out, ce_mppi_info* info,
                                   hipStream_t s) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  if (!x_t || !u_out) return fail(CE_EINVAL, "x_t and u_out must not be NULL");
  if (n_obs < 0 || n_obs > P->c.max_obs) return fail(CE_EINVAL, "n_obs outside 0..max_obstacles");
  if (n_obs > 0 && !obstacles) return fail(CE_EINVAL, "obstacles is NULL with n_obs > 0");
  DeviceGuard guard(P->cfg.device);
  mark_stream(P, s);
  Timing& t = P->t;
  hipError_t e = hipSuccess;
  if (t.cap > 0 && t.n < t.cap) {
    // timed replan: direct launches between events
    const int i = t.n++;
    Launcher L(s);
    e = hipEventRecord(t.ev[3 * i], s);
    launch_rollout(L, P->c, P->b, x_t, obstacles, n_obs);
    if (e == hipSuccess && L.err == hipSuccess) e = hipEventRecord(t.ev[3 * i + 1], s);
    launch_post_rollout(L, P->c, P->b);
    launch_finish(L, P->c, P->b, u_out, U_out, info);
    if (e == hipSuccess && L.err == hipSuccess) e = hipEventRecord(t.ev[3 * i + 2], s);
    if (e == hipSuccess) e = L.err;
  } else if (P->launch_mode == CE_LAUNCH_GRAPH) {
    e = replan_graph(P, x_t, obstacles, n_obs, u_out, U_out, info, s);
  } else {
    Launcher L(s);
    launch_rollout(L, P->c, P->b, x_t, obstacles, n_obs);
    launch_post_rollout(L, P->c, P->b);
    launch_finish(L, P->c, P->b, u_out, U_out, info);
    e = L.err;
  }
  if (e != hipSuccess) return hip_fail(e, "replan launch");
  return CE_OK;
}
}  // namespace cemppi

extern "C" {

ce_status ce_mppi_replan(ce_mppi_planner* P, const float* x_t, const float* obstacles, int32_t n_obs,
                         float* u_out, float* U_out, ce_mppi_info* info, void* stream) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  DeviceGuard guard(P->cfg.device);
  const ce_status st = check_not_busy(P, S(stream));
  if (st != CE_OK) return st;
  return replan_unchecked(P, x_t, obstacles, n_obs, u_out, U_out, info, S(stream));
}


ce_status ce_mppi_set_dbscan_mode(ce_mppi_planner* P, int32_t mode) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  Cfg& c = P->c;
  int path;
  switch (mode) {
    case CE_DBSCAN_AUTO: path = P->b.wcnt ? 0 : (P->b.adj ? 1 : 2); break;
    case CE_DBSCAN_WINDOW:
      if (!P->b.wcnt)
        return fail(CE_EUNSUPPORTED, "angular windows need 2-D features and eps in [0.01, 1.4]");
      path = 0;
      break;
    case CE_DBSCAN_BITMAP:
      if (!P->b.adj) return fail(CE_EUNSUPPORTED, "the eps-adjacency bitmap needs K <= 16384");
      path = 1;
      break;
    case CE_DBSCAN_TILED: path = 2; break;
    default: return fail(CE_EINVAL, "unknown DBSCAN mode");
  }
  if (path != c.dbpath) {
    DeviceGuard guard(P->cfg.device);
    drop_graph(P->g);  // the recorded chain holds the previous path's kernels
    c.dbpath = path;
  }
  return CE_OK;
}

ce_status ce_mppi_get_dbscan_path(const ce_mppi_planner* P, int32_t* path) {
  if (!P || !path) return fail(CE_EINVAL, "planner or path is NULL");
  *path = P->c.dbpath == 0 ? CE_DBSCAN_WINDOW : (P->c.dbpath == 1 ? CE_DBSCAN_BITMAP : CE_DBSCAN_TILED);
  return CE_OK;
}

ce_status ce_mppi_set_launch_mode(ce_mppi_planner* P, int32_t mode) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  if (mode != CE_LAUNCH_GRAPH && mode != CE_LAUNCH_DIRECT) return fail(CE_EINVAL, "unknown launch mode");
  P->launch_mode = mode;
  return CE_OK;
}

ce_status ce_mppi_timing_enable(ce_mppi_planner* P, int32_t capacity) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  if (capacity < 0 || capacity > (1 << 20)) return fail(CE_EINVAL, "capacity out of range");
  DeviceGuard guard(P->cfg.device);
  drop_timing(P->t);
  if (capacity == 0) return CE_OK;
  P->t.ev.resize((size_t)capacity * 3, nullptr);
  for (auto& ev : P->t.ev) {
    hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      drop_timing(P->t);
      return hip_fail(e, "hipEventCreate");
    }
  }
  P->t.cap = capacity;
  P->t.n = 0;
  return CE_OK;
}

ce_status ce_mppi_timing_read(ce_mppi_planner* P, double* rollout_ms, double* post_ms,
                              double* total_ms, int32_t* count) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  DeviceGuard guard(P->cfg.device);
  const Timing& t = P->t;
  double r = 0.0, q = 0.0, a = 0.0;
  for (int i = 0; i < t.n; ++i) {
    hipError_t e = hipEventSynchronize(t.ev[3 * i + 2]);
    float x = 0.f, y = 0.f, z = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&x, t.ev[3 * i], t.ev[3 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&y, t.ev[3 * i + 1], t.ev[3 * i + 2]);
    if (e == hipSuccess) e = hipEventElapsedTime(&z, t.ev[3 * i], t.ev[3 * i + 2]);
    if (e != hipSuccess) return hip_fail(e, "timing_read");
    r += x;
    q += y;
    a += z;
  }
  if (rollout_ms) *rollout_ms = r;
  if (post_ms) *post_ms = q;
  if (total_ms) *total_ms = a;
  if (count) *count = t.n;
  return CE_OK;
}

ce_status ce_mppi_timing_read_each(ce_mppi_planner* P, int32_t cap, double* rollout_ms,
                                   double* post_ms, double* total_ms, int32_t* count) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  if (cap < 0 || (cap > 0 && (!rollout_ms || !post_ms || !total_ms)))
    return fail(CE_EINVAL, "bad output arrays");
  DeviceGuard guard(P->cfg.device);
  const Timing& t = P->t;
  const int n = t.n < cap ? t.n : cap;
  for (int i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(t.ev[3 * i + 2]);
    float x = 0.f, y = 0.f, z = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&x, t.ev[3 * i], t.ev[3 * i + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&y, t.ev[3 * i + 1], t.ev[3 * i + 2]);
    if (e == hipSuccess) e = hipEventElapsedTime(&z, t.ev[3 * i], t.ev[3 * i + 2]);
    if (e != hipSuccess) return hip_fail(e, "timing_read_each");
    rollout_ms[i] = x;
    post_ms[i] = y;
    total_ms[i] = z;
  }
  if (count) *count = t.n;
  return CE_OK;
}

ce_status ce_mppi_time_rollout(ce_mppi_planner* P, const float* x_t, const float* obstacles,
                               int32_t n_obs, int32_t reps, void* stream, double* ms_per_launch) {
  if (!P || !x_t || !ms_per_launch) return fail(CE_EINVAL, "NULL argument");
  if (reps < 1 || reps > 100000) return fail(CE_EINVAL, "reps out of range");
  if (n_obs < 0 || n_obs > P->c.max_obs) return fail(CE_EINVAL, "n_obs out of range");
  if (n_obs > 0 && !obstacles) return fail(CE_EINVAL, "obstacles is NULL");
  size_t need = 0;
  ce_status st = ce_mppi_state_size(P, &need);
  if (st != CE_OK) return st;
  std::vector<char> saved(need);
  st = ce_mppi_get_state(P, saved.data(), need, stream);
  if (st != CE_OK) return st;
  DeviceGuard guard(P->cfg.device);
  hipStream_t s = S(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  Launcher L(s);
  for (int i = 0; i < reps && e == hipSuccess && L.err == hipSuccess; ++i)
    launch_rollout(L, P->c, P->b, x_t, obstacles, n_obs);
  if (e == hipSuccess) e = L.err;
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "time_rollout");
  *ms_per_launch = (double)ms / reps;
  // the rollout phase pushes the observation into the history ring: put the
  // saved state back
  return ce_mppi_set_state(P, saved.data(), need, stream);
}

ce_status ce_mppi_tune_launch(ce_mppi_planner* P, const float* x_t, const float* obstacles,
                              int32_t n_obs, float* u_out, int32_t reps, void* stream,
                              double* us_graph, double* us_direct) {
  if (!P || !x_t || !u_out) return fail(CE_EINVAL, "NULL argument");
  if (reps < 1 || reps > 10000) return fail(CE_EINVAL, "reps out of range");
  if (n_obs < 0 || n_obs > P->c.max_obs) return fail(CE_EINVAL, "n_obs out of range");
  if (n_obs > 0 && !obstacles) return fail(CE_EINVAL, "obstacles is NULL");
  size_t need = 0;
  ce_status st = ce_mppi_state_size(P, &need);
  if (st != CE_OK) return st;
  std::vector<char> saved(need);
  st = ce_mppi_get_state(P, saved.data(), need, stream);
  if (st != CE_OK) return st;
  DeviceGuard guard(P->cfg.device);
  hipStream_t s = S(stream);
  const int keep_cap = P->t.cap;
  P->t.cap = 0;  // the timed mode would bypass the launch mode under test
  double us[2] = {0.0, 0.0};
  const int32_t modes[2] = {CE_LAUNCH_GRAPH, CE_LAUNCH_DIRECT};
  for (int m = 0; m < 2 && st == CE_OK; ++m) {
    P->launch_mode = modes[m];
    // one untimed replan (builds the graph), then `reps` back to back: host
    // wall time from the first call to the stream being idle, which counts
    // whichever of host submission and device work is the bottleneck
    st = ce_mppi_replan(P, x_t, obstacles, n_obs, u_out, nullptr, nullptr, stream);
    if (st == CE_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(CE_EDEVICE, "tune_launch sync");
    const auto t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < reps && st == CE_OK; ++i)
      st = ce_mppi_replan(P, x_t, obstacles, n_obs, u_out, nullptr, nullptr, stream);
    if (st == CE_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(CE_EDEVICE, "tune_launch sync");
    const auto t1 = std::chrono::steady_clock::now();
    us[m] = std::chrono::duration<double, std::micro>(t1 - t0).count() / reps;
    if (st == CE_OK) st = ce_mppi_set_state(P, saved.data(), need, stream);
  }
  P->t.cap = keep_cap;
  if (st != CE_OK) return st;
  P->launch_mode = us[1] < us[0] ? CE_LAUNCH_DIRECT : CE_LAUNCH_GRAPH;
  if (us_graph) *us_graph = us[0];
  if (us_direct) *us_direct = us[1];
  return CE_OK;
}

ce_status ce_mppi_replan_from_rollouts(ce_mppi_planner* P, const float* x_t, const float* obstacles,
                                       int32_t n_obs, const float* S_in, const int32_t* collide,
                                       const int32_t* first_obs, const float* p_term,
                                       const float* p_first, const float* eps, float* u_out,
                                       float* U_out, ce_mppi_info* info, void* stream) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  if (!x_t || !u_out || !S_in || !collide || !first_obs || !p_term || !p_first || !eps)
    return fail(CE_EINVAL, "NULL input or output");
  if (n_obs < 0 || n_obs > P->c.max_obs) return fail(CE_EINVAL, "n_obs outside 0..max_obstacles");
  if (n_obs > 0 && !obstacles) return fail(CE_EINVAL, "obstacles is NULL with n_obs > 0");
  DeviceGuard guard(P->cfg.device);
  const Cfg& c = P->c;
  const Bufs& b = P->b;
  const size_t K = (size_t)c.K;
  hipStream_t s = S(stream);
  ce_status busy = check_not_busy(P, s);
  if (busy != CE_OK) return busy;
  mark_stream(P, s);
  hipError_t e = hipMemcpyAsync(b.S, S_in, K * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b.col, collide, K * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b.first, first_obs, K * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b.pT, p_term, K * c.p * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b.pF, p_first, K * c.p * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b.eps, eps, K * c.NM * 4, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "replan_from_rollouts copy");
  Launcher L(s);
  launch_reduce_records(L, c, b, x_t, obstacles, n_obs);
  launch_post_rollout(L, c, b);
  launch_finish(L, c, b, u_out, U_out, info);
  if (L.err != hipSuccess) return hip_fail(L.err, "replan_from_rollouts");
  return CE_OK;
}

ce_status ce_mppi_stage_dbscan(ce_mppi_planner* P, const float* z, int32_t V, int32_t* ncount,
                               int32_t* label, int32_t* n_clusters, void* stream) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  if (V < 0 || (size_t)V > P->cap_K) return fail(CE_EINVAL, "V outside 0..K");
  if (V > 0 && (!z || !label)) return fail(CE_EINVAL, "z and label must not be NULL");
  DeviceGuard guard(P->cfg.device);
  const Cfg& c = P->c;
  const Bufs& b = P->b;
  hipStream_t s = S(stream);
  hipError_t e = hipSuccess;
  const float* zin = z;
  if (V > 0 && c.p == 3) {
    // caller layout [V][3] -> internal float4 rows
    e = hipMemcpy2DAsync(b.gv, 16, z, 12, 12, V, hipMemcpyDeviceToDevice, s);
    zin = b.gv;
  }
  if (e != hipSuccess) return hip_fail(e, "stage_dbscan copy");
  Launcher L(s);
  launch_stage_dbscan(L, c, b, zin, V, ncount, label, n_clusters);
  if (L.err != hipSuccess) return hip_fail(L.err, "stage_dbscan");
  return CE_OK;
}

ce_status ce_mppi_stage_noise(ce_mppi_planner* P, uint32_t step, uint32_t* words, float* gauss,
                              void* stream) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  DeviceGuard guard(P->cfg.device);
  Launcher L(S(stream));
  launch_stage_noise(L, P->c, step, words, gauss);
  if (L.err != hipSuccess) return hip_fail(L.err, "stage_noise");
  return CE_OK;
}

ce_status ce_mppi_set_nominal(ce_mppi_planner* P, const float* U, void* stream) {
  if (!P || !U) return fail(CE_EINVAL, "NULL argument");
  DeviceGuard guard(P->cfg.device);
  hipError_t e = hipMemcpyAsync(P->b.U, U, (size_t)P->c.NM * 4, hipMemcpyDeviceToDevice, S(stream));
  if (e != hipSuccess) return hip_fail(e, "set_nominal");
  return CE_OK;
}

ce_status ce_mppi_get_nominal(const ce_mppi_planner* P, float* U, void* stream) {
  if (!P || !U) return fail(CE_EINVAL, "NULL argument");
  DeviceGuard guard(P->cfg.device);
  hipError_t e = hipMemcpyAsync(U, P->b.U, (size_t)P->c.NM * 4, hipMemcpyDeviceToDevice, S(stream));
  if (e != hipSuccess) return hip_fail(e, "get_nominal");
  return CE_OK;
}

namespace {
// persistent part of the control block
struct Persist {
  uint32_t step_lo, step_hi;
  int32_t hist_head, hist_count, hist_nobs;
};
static_assert(offsetof(Ctrl, step_lo) == 0 && offsetof(Ctrl, hist_nobs) == 16, "Ctrl prefix");

struct StateHeader {
  uint32_t magic, abi, dyn, N, m, p, H, max_obs;
};
constexpr uint32_t kStateMagic = 0x43454d50u;  // "CEMP"

// writes the persistent prefix and sets the start-of-replan ring snapshot to
// the same ring state
ce_status write_persist(ce_mppi_planner* P, const Persist& ps, hipStream_t s) {
  struct {
    Persist p;
    int32_t hs_head, hs_count, hs_nobs;
  } w{ps, ps.hist_head, ps.hist_count, ps.hist_nobs};
  static_assert(offsetof(Ctrl, hs_head) == sizeof(Persist) && sizeof(w) == offsetof(Ctrl, n_obs),
                "Ctrl snapshot follows the persistent prefix");
  hipError_t e = hipMemcpyAsync(P->b.ctrl, &w, sizeof(w), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "control block update");
  return CE_OK;
}

ce_status read_persist(const ce_mppi_planner* P, Persist& ps, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(&ps, P->b.ctrl, sizeof(ps), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "control block read");
  return CE_OK;
}

size_t hist_floats(const Cfg& c) {
  return (size_t)c.H * (size_t)(c.max_obs > 0 ? c.max_obs : 1) * (size_t)c.p;
}
}  // namespace

ce_status ce_mppi_reset_history(ce_mppi_planner* P, void* stream) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  DeviceGuard guard(P->cfg.device);
  Persist ps;
  ce_status st = read_persist(P, ps, S(stream));
  if (st != CE_OK) return st;
  ps.hist_head = P->c.H - 1;
  ps.hist_count = 0;
  ps.hist_nobs = -1;
  return write_persist(P, ps, S(stream));
}

ce_status ce_mppi_set_history(ce_mppi_planner* P, const float* hist, int32_t h_count, int32_t n_obs,
                              void* stream) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  const Cfg& c = P->c;
  if (h_count < 0 || n_obs < 0 || n_obs > c.max_obs)
    return fail(CE_EINVAL, "h_count must be >= 0 and n_obs within 0..max_obstacles");
  if (h_count > 0 && n_obs > 0 && !hist) return fail(CE_EINVAL, "hist is NULL");
  DeviceGuard guard(P->cfg.device);
  hipStream_t s = S(stream);
  const int keep = h_count < c.H ? h_count : c.H;
  // entry i (0 = newest) goes to ring slot head - i
  const int head = keep > 0 ? keep - 1 : c.H - 1;
  const size_t row = (size_t)n_obs * c.p;
  hipError_t e = hipSuccess;
  for (int i = 0; i < keep && row > 0 && e == hipSuccess; ++i) {
    const int slot = ((head - i) % c.H + c.H) % c.H;
    e = hipMemcpyAsync(P->b.hist + (size_t)slot * c.max_obs * c.p, hist + (size_t)i * row,
                       row * sizeof(float), hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) return hip_fail(e, "set_history");
  Persist ps;
  ce_status st = read_persist(P, ps, s);
  if (st != CE_OK) return st;
  ps.hist_head = head;
  ps.hist_count = keep;
  ps.hist_nobs = keep > 0 ? n_obs : -1;
  return write_persist(P, ps, s);
}

ce_status ce_mppi_set_step(ce_mppi_planner* P, uint64_t step, void* stream) {
  if (!P) return fail(CE_EINVAL, "planner is NULL");
  DeviceGuard guard(P->cfg.device);
  Persist ps;
  ce_status st = read_persist(P, ps, S(stream));
  if (st != CE_OK) return st;
  ps.step_lo = (uint32_t)(step & 0xffffffffu);
  ps.step_hi = (uint32_t)(step >> 32);
  return write_persist(P, ps, S(stream));
}

ce_status ce_mppi_state_size(const ce_mppi_planner* P, size_t* bytes) {
  if (!P || !bytes) return fail(CE_EINVAL, "NULL argument");
  *bytes = sizeof(StateHeader) + sizeof(Persist) + (size_t)P->c.NM * 4 + hist_floats(P->c) * 4;
  return CE_OK;
}

ce_status ce_mppi_get_state(const ce_mppi_planner* P, void* buf, size_t bytes, void* stream) {
  size_t need = 0;
  ce_status st = ce_mppi_state_size(P, &need);
  if (st != CE_OK) return st;
  if (!buf || bytes < need) return fail(CE_EINVAL, "state buffer too small");
  DeviceGuard guard(P->cfg.device);
  char* out = static_cast<char*>(buf);
  StateHeader h{kStateMagic, CE_MPPI_ABI_VERSION, (uint32_t)P->c.dyn, (uint32_t)P->c.N,
                (uint32_t)P->c.m, (uint32_t)P->c.p, (uint32_t)P->c.H, (uint32_t)P->c.max_obs};
  std::memcpy(out, &h, sizeof(h));
  Persist ps;
  st = read_persist(P, ps, S(stream));
  if (st != CE_OK) return st;
  std::memcpy(out + sizeof(h), &ps, sizeof(ps));
  char* p = out + sizeof(h) + sizeof(ps);
  hipError_t e = hipMemcpyAsync(p, P->b.U, (size_t)P->c.NM * 4, hipMemcpyDeviceToHost, S(stream));
  if (e == hipSuccess)
    e = hipMemcpyAsync(p + (size_t)P->c.NM * 4, P->b.hist, hist_floats(P->c) * 4,
                       hipMemcpyDeviceToHost, S(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
  if (e != hipSuccess) return hip_fail(e, "get_state");
  return CE_OK;
}

ce_status ce_mppi_set_state(ce_mppi_planner* P, const void* buf, size_t bytes, void* stream) {
  size_t need = 0;
  ce_status st = ce_mppi_state_size(P, &need);
  if (st != CE_OK) return st;
  if (!buf || bytes < need) return fail(CE_EINVAL, "state buffer too small");
  const char* in = static_cast<const char*>(buf);
  StateHeader h;
  std::memcpy(&h, in, sizeof(h));
  if (h.magic != kStateMagic || h.abi != CE_MPPI_ABI_VERSION || h.dyn != (uint32_t)P->c.dyn ||
      h.N != (uint32_t)P->c.N || h.m != (uint32_t)P->c.m || h.p != (uint32_t)P->c.p ||
      h.H != (uint32_t)P->c.H || h.max_obs != (uint32_t)P->c.max_obs)
    return fail(CE_EINVAL, "state was saved by a planner with a different configuration");
  DeviceGuard guard(P->cfg.device);
  Persist ps;
  std::memcpy(&ps, in + sizeof(h), sizeof(ps));
  const char* p = in + sizeof(h) + sizeof(ps);
  hipError_t e = hipMemcpyAsync(P->b.U, p, (size_t)P->c.NM * 4, hipMemcpyHostToDevice, S(stream));
  if (e == hipSuccess)
    e = hipMemcpyAsync(P->b.hist, p + (size_t)P->c.NM * 4, hist_floats(P->c) * 4,
                       hipMemcpyHostToDevice, S(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
  if (e != hipSuccess) return hip_fail(e, "set_state");
  return write_persist(P, ps, S(stream));
}

ce_status ce_mppi_debug_get(const ce_mppi_planner* P, int32_t which, void* dst, size_t bytes,
                            void* stream) {
  if (!P || !dst) return fail(CE_EINVAL, "NULL argument");
  DeviceGuard guard(P->cfg.device);
  const Cfg& c = P->c;
  const Bufs& b = P->b;
  const size_t K = (size_t)c.K, p = (size_t)c.p;
  const void* src = nullptr;
  size_t cap = 0;
  size_t rows = 0, src_pitch = 0;  // strided float4 rows (p = 3 features)
  switch (which) {
    case CE_DBG_COST: src = b.S; cap = K * 4; break;
    case CE_DBG_COLLIDE: src = b.col; cap = K * 4; break;
    case CE_DBG_FIRST_OBS: src = b.first; cap = K * 4; break;
    case CE_DBG_P_TERM: src = b.pT; cap = K * p * 4; break;
    case CE_DBG_P_FIRST: src = b.pF; cap = K * p * 4; break;
    case CE_DBG_EPS: src = b.eps; cap = K * (size_t)c.NM * 4; break;
    case CE_DBG_V_IDX: src = b.vidx; cap = K * 4; break;
    case CE_DBG_Z: src = b.z; cap = K * p * 4; if (p == 3) { rows = K; src_pitch = 16; } break;
    case CE_DBG_G: src = b.gv; cap = K * p * 4; if (p == 3) { rows = K; src_pitch = 16; } break;
    case CE_DBG_NCOUNT: src = b.ncount; cap = K * 4; break;
    case CE_DBG_LABEL: src = b.label; cap = K * 4; break;
    case CE_DBG_CLUSTER_COST: src = b.c_cost; cap = (size_t)c.mcap * 4; break;
    case CE_DBG_CLUSTER_DIR: src = b.c_dir; cap = (size_t)c.mcap * p * 4; rows = c.mcap; src_pitch = 16; break;
    case CE_DBG_CLUSTER_SIZE: src = b.c_size; cap = (size_t)c.mcap * 4; break;
    case CE_DBG_TREES: src = &b.ctrl->n_trees; cap = 8; break;
    default: return fail(CE_EINVAL, "unknown debug buffer");
  }
  const size_t n = bytes < cap ? bytes : cap;
  hipError_t e;
  if (src_pitch) {
    const size_t row_bytes = p * 4;
    const size_t nrows = n / row_bytes < rows ? n / row_bytes : rows;
    e = nrows ? hipMemcpy2DAsync(dst, row_bytes, src, src_pitch, row_bytes, nrows,
                                 hipMemcpyDeviceToDevice, S(stream))
              : hipSuccess;
  } else {
    e = hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, S(stream));
  }
  if (e != hipSuccess) return hip_fail(e, "debug_get");
  return CE_OK;
}

const char* ce_mppi_status_string(ce_status s) {
  switch (s) {
    case CE_OK: return "ok";
    case CE_EINVAL: return "invalid argument";
    case CE_ENOMEM: return "out of device memory";
    case CE_EDEVICE: return "device error";
    case CE_EUNSUPPORTED: return "unsupported";
    case CE_EBUSY: return "busy";
    default: return "unknown status";
  }
}

const char* ce_mppi_last_error(void) { return g_err.c_str(); }

}  // extern "C"
