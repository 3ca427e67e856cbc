// device.hpp -- data layout and device primitives of the CE-MPPI replan
// kernels for gfx950 (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cemppi {

constexpr int kMaxCtrl = 6;
constexpr int kMaxObs = 64;
constexpr int kMaxHorizon = 63;
constexpr int kMaxHistory = 16;
constexpr int kMaxSpheres = 16;
constexpr int kMaxNM = kMaxHorizon * kMaxCtrl;
constexpr int kWave = 64;

// rollout kernel: 512 threads = 8 waves; a wave holds one rollout (64-lane
// segment) or two (32-lane segments) when N + 1 <= 32.
constexpr int kRollThreads = 512;
constexpr int kRollWaves = kRollThreads / 64;
constexpr int kMaxRpb = 2 * kRollWaves;  // rollouts per block at one round per wave
constexpr int kMaxR = 8;                 // rollout rounds per wave (batched form)
constexpr int kGroup = 8;                // rollouts per partial record
// per-block partial record of the rollout reduction (floats)
constexpr int kPart = 12;
enum PartField {
  P_NCOL = 0, P_NREF = 1, P_NFEAS = 2, P_SMIN_ALL = 3, P_SMIN_FEAS = 4,
  P_SUM_REF = 5,   // 3 floats: sum over colliding rollouts that hit o*
  P_SUM_COL = 8,   // 3 floats: sum over every colliding rollout
};

// DBSCAN tiles: kTile rows (one per thread) x kTile columns (staged in LDS)
constexpr int kTile = 128;
// update kernel: candidates per block (16 per wave) and threads; the
// single-block finisher
constexpr int kUpdChunk = 64;
constexpr int kUpdThreads = 256;
constexpr int kFinThreads = 1024;
static_assert(kMaxNM <= kFinThreads, "the final combination holds one element per thread");
// tree graph handled by the fast path
constexpr int kMaxTrees = 64;
constexpr int kColGroup = 2;   // column tiles per tree-adjacency block
constexpr int kCntGroup = 2;   // column tiles per count / core-neighbour block (early exit)
constexpr int kSplit = 4;       // threads per row in the tiled passes of small single planners
constexpr int kSplitTiles = 32; // planners of at most this many tiles use them
constexpr int kSortBins = 4096; // Morton cells of the DBSCAN spatial order
// eps-adjacency bitmap of the single-planner DBSCAN: planners of at most
// kAdjMaxK rollouts keep one (ceil(K/kTile)^2 * kTile * 16 bytes: 8 MiB at
// K = 8192, 32 MiB at the limit); larger ones use the distance passes
constexpr int kAdjMaxK = 16384;
constexpr int kAdjGroup = 1;       // column tiles per bitmap block
constexpr int kMcnThreads = 1024;  // core-neighbour pass on the bitmap: 64 rows per block
constexpr int kMcnSplit = kMcnThreads / 64;  // threads per row there
constexpr int kMcnLoads = (kAdjMaxK / kTile + kMcnSplit - 1) / kMcnSplit;  // row words per thread
// angular-window DBSCAN of single planners with 2-D features (the unit
// directions of Eq. (13)): points on the unit ring are binned by angle into
// kWinBins buckets; the compacted index of a point and its slot in its bucket
// share one key (bucket << kWinShift | slot), so V <= 2^kWinShift, which
// covers every planner size
constexpr int kWinBins = 4096;
constexpr int kWinShift = 16;
constexpr int kWinMaxK = 1 << kWinShift;
constexpr int kWinMaxRuns = 1024;  // runs of core buckets (at most kWinBins / (gap + 1) with gap >= 3)
constexpr int kWinPos = 512;  // sorted positions per count-and-place block
static_assert(kWinMaxK >= kAdjMaxK, "the windowed path covers every planner with a bitmap");
constexpr int kLabBatch = 8;   // points per thread per labelling pass
constexpr int kRecBatch = 4;   // partial records per thread in flight at once
constexpr int kFinRows = 8;    // update-partial rows per wave in flight at once (final combination)
constexpr int kFinChunks = (kMaxNM + 1 + 63) / 64;  // 64-element chunks of a partial row, at most
constexpr int kStatClusters = 64;  // clusters per statistics pass of the labelling block

constexpr int kInt32Max = 0x7fffffff;

// Device control block of one planner: per-replan decisions shared between
// kernels plus the persistent counters.
struct Ctrl {
  // persistent
  uint32_t step_lo, step_hi;
  int32_t hist_head, hist_count, hist_nobs;
  // the ring state at the start of the replan (copied by the last kernel of
  // each replan): the rollout blocks read it while block 0 pushes the new
  // observation
  int32_t hs_head, hs_count, hs_nobs;
  // per replan
  int32_t n_obs, nonfinite, closest;
  int32_t n_col, n_feas, n_ref, branch;
  float p0[3];
  float ref[3];
  float smin_all, smin_feas;
  int32_t n_trees, tree_overflow, M;
  int32_t sel, sel_size, rule, h_used;
  float margin, smin_sel, wsum;
  float v_obs[3], v_hat[3];
  int32_t dyn_h, dyn_ok;  // Eq. (17) estimate of this replan: H' and whether the dynamic rule applies
  uint32_t status;
  uint32_t step_used;
  int32_t wticket;  // completion ticket of the window DBSCAN launch (zero between calls)
};

// Scalar configuration (kernel argument).
struct Cfg {
  int dyn, N, K, m, n, p, NM, B;
  int seg, rpb, nblk_roll;
  int roll_r;       // rollout rounds per wave of the single-planner launch (1 or 2)
  int npart;        // ceil(K / kGroup) partial records
  float dt, lambda, norm_eps;
  float L[36];
  float umin[6], umax[6];
  float eps2;
  int min_pts;
  int scene_mode, H;
  float v_obs_min;
  int ref_mode, max_obs;
  float robot_r;
  float reach;      // unicycle: bound on |p(x_j) - p(x_t)|, max|v| N dt (infinite: no bound)
  float goal[6], Q[6], R[6], Qf[6];
  float dh_a[6], dh_d[6], dh_ca[6], dh_sa[6], dh_off[6];
  int ns;
  float rs;
  int sph_seg[kMaxSpheres];
  float sph_t[kMaxSpheres];
  float qlim[6], wlim;
  int pose;        // arm: pose cost of the real-robot experiment
  int cv;          // obstacles move with constant velocity inside the rollouts
  float Rg[9];     // pose cost: goal orientation, row-major
  uint32_t seed_lo, seed_hi, stream_id;
  int ntile;       // ceil(K / kTile)
  int nblk_upd;    // update kernel blocks
  int mcap;        // cluster capacity
  // DBSCAN path: 0 angular windows, 1 eps-adjacency bitmap, 2 distance passes
  int dbpath;
  // angular windows (dbpath 0): bucket coordinate u = (atan2(z) + pi) * w_scale;
  // ring points have |z|^2 in [w_r2lo, w_r2hi]; from a point at u, every ring
  // point of the buckets inside u +- w_in is a neighbour and none outside
  // u +- w_out is; occupied buckets at most w_g apart are linked for certain,
  // more than w_gout apart never
  float w_scale, w_in, w_out, w_r2lo, w_r2hi;
  int w_g, w_gout;
};

// Device buffers of one planner (kernel argument).
struct Bufs {
  Ctrl* ctrl;
  float* U;        // [N][m] nominal sequence
  float* hist;     // [H][max_obs][p] ring of obstacle centres
  // per rollout
  float* S;        // [K]
  int* col;        // [K]
  int* first;      // [K]
  float* pT;       // [K][p]
  float* pF;       // [K][p]
  float* g;        // [K][p]
  float* eps;      // [K][N][m]
  float* part;     // [npart (+ slack)][kPart] rollout-group partial records
  // compacted feasible set
  int* vidx;       // [K]
  float* z;        // [K][zs] zs = 2 (p = 2) or 4 (p = 3)
  float* gv;       // [K][zs]
  float* Sv;       // [K]
  // DBSCAN
  float* zs;       // [K][zs] features in Morton order
  int* sid;        // [K] original index of each sorted position
  float4* tlo;     // [ntile] lower corner of each sorted tile's box
  float4* thi;     // [ntile] upper corner
  int* ncount;     // [K]
  int* mcn;        // [K] lowest-index core neighbour (kInt32Max if none)
  int* root;       // [K] tree root (core points), -1 otherwise
  unsigned long long* tadj;     // [kMaxTrees] tree adjacency rows (OR of every tree-adjacency block)
  uint4* adj;      // [ntile][ntile * kTile] eps-adjacency words (null: distance passes)
  int* label;      // [K]
  unsigned long long* coremask;  // [ceil(K/64)] core flags
  unsigned long long* hookmask;  // [ceil(K/64)] core neighbour of lower index found
  // cluster statistics
  float* c_cost;   // [mcap] mean cost
  float* c_dir;    // [mcap][4] normalised mean direction
  int* c_size;     // [mcap]
  float* c_smin;   // [mcap]
  // update partials
  // angular-window DBSCAN (null unless the planner has p = 2 and K <= kWinMaxK);
  // the sorted features and their indices use zs and sid
  int* wcnt;       // [kWinBins + 1] points per bucket (the last: off the ring); zero between calls
  int* wstart;     // [kWinBins + 2] first sorted position of each bucket; [kWinBins] = ring points
  int* wkey;       // [K] bucket << kWinShift | slot, by compacted index
  int* wbmin;      // [kWinBins] kWinMaxK - lowest core index in each bucket (0 if none); zero between calls
  int* wnc;        // [K] neighbour counts by sorted position
  int* wuf;        // [3][kWinMaxRuns + K] union-find parents, component minima, off-ring labels
  int* wzone;      // [ceil(K / kWinPos)][K] indices of a count block's zone when it exceeds LDS
  float* upart;    // [nblk_upd][NM + 1]
  float* Unew;     // [N][m] updated sequence before the shift
};

// ---------------------------------------------------------------------------
// Batched execution: many planners per launch.  Each planner of a batch has a
// slot: its configuration and buffers (written at batch creation) and its
// per-call inputs and outputs.  Kernels read slots through constant-address
// pointers, so every field is a scalar load as with a kernel argument.
constexpr int kMaxBatch = 1024;   // planners per batch

struct SlotStatic {
  Cfg c;
  Bufs b;
};
struct SlotIO {
  const float* x_t;
  const float* obs;
  float* u_out;
  float* U_out;
  void* info;
  int n_obs;
  int pad;
};
typedef const __attribute__((address_space(4))) SlotStatic* CSlotStatic;
typedef const __attribute__((address_space(4))) SlotIO* CSlotIO;

// Work table of one phase over one group of planners: slot[q] is the slot of
// the q-th planner, pref[0..n] the exclusive prefix of its work items; the
// count n is read from device memory, so one graph serves any member subset.
struct Tab {
  const int* slot;
  const int* pref;
  const int* n;
};

// Persistent loop over the items of a table: block i takes items i, i +
// gridDim.x, ...; f(slot, local item) runs with every thread of the block
// (NT threads: a compile-time block size, so the kernel does not read the
// dispatch packet for it).
template <int NT, typename F>
__device__ __forceinline__ void for_each_item(const Tab& t, int* s_pref, F&& f) {
  const int n = __builtin_amdgcn_readfirstlane(*t.n);
  for (int i = threadIdx.x; i <= n; i += NT) s_pref[i] = t.pref[i];
  __syncthreads();
  const int total = s_pref[n];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    // the planner of item it: the last q with pref[q] <= it
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_pref[mid] <= it) lo = mid;
      else hi = mid - 1;
    }
    const int q = __builtin_amdgcn_readfirstlane(lo);
    const int slot = __builtin_amdgcn_readfirstlane(t.slot[q]);
    f(slot, it - s_pref[q]);
    __syncthreads();
  }
}

// Tables of the batched post-rollout phases.  Index kd is the group of
// planners: p = 2 on the sorted distance passes (0), p = 3 (1), p = 2 on the
// angular windows (2).  Static tables for compaction and for the tree
// closure, components and statistics (one item per planner); the DBSCAN
// tables are filled on the device from each planner's feasible count
// (PlanOut).  Update and finish run over every planner of the batch.
constexpr int kPlanKinds = 3;
struct PlanOut {
  const int* slot[kPlanKinds];  // planners of each group
  const int* n[kPlanKinds];     // their counts (device memory)
  int* pref_cnt[kPlanKinds];    // count and lowest-core-neighbour tiles (group 2: count blocks)
  int* pref_adj[kPlanKinds];    // tree-adjacency tiles
  int colg;                     // column tiles per count/mcn item
};

struct BatchTabs {
  Tab compact[kPlanKinds], cnt[kPlanKinds], adj[kPlanKinds], cc[kPlanKinds];
  Tab update, finish;
  PlanOut plan;
  int grid_compact[kPlanKinds], grid_cc[kPlanKinds], grid_update, grid_finish;
  int grid_tile, grid_win;
  int colg;
  int has[kPlanKinds];  // the batch has planners of the group (its phases are launched)
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, key bumped by
// the Weyl constants between rounds.
__device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32x32 -> 64-bit product each (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// open-interval uniform (2*(w>>9)+1) * 2^-24, exact in FP32
__device__ __forceinline__ float u01(uint32_t w) {
  return (float)(((w >> 9) << 1) | 1u) * 5.9604644775390625e-8f;
}

// Box-Muller pair on the hardware transcendentals: r = sqrt(-2 ln u_a) with
// ln u = ln 2 * log2 u (v_log_f32, v_sqrt_f32), and the angle 2 pi u_b taken
// by v_cos_f32 / v_sin_f32, whose argument is in revolutions.  Measured
// against FP64 over 4M pairs: max |d| / max(|g|, 1) = 3.2e-7 (the library
// sqrtf/logf/sincospif path: 2.3e-7), at a fraction of the instructions.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& ga, float& gb) {
  const float r = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u01(wa)));
  const float t = u01(wb);
  ga = r * __builtin_amdgcn_cosf(t);
  gb = r * __builtin_amdgcn_sinf(t);
}

// Standard normals g[0..M) of step j of rollout k: elements j*M .. j*M+M-1 of
// the flattened sequence; element pair q (elements 2q, 2q+1) is the
// Box-Muller pair of words (0,1) of counter block q/2 when q is even and of
// words (2,3) when q is odd.  Straight-line code for the two control sizes.
template <int M>
__device__ __forceinline__ void step_gaussians(const Cfg& c, uint32_t step, int k, int j, float* g);

template <>
__device__ __forceinline__ void step_gaussians<2>(const Cfg& c, uint32_t step, int k, int j, float* g) {
  // pair q = j: block j/2, half j&1
  uint32_t w[4];
  philox((uint32_t)(j >> 1), (uint32_t)k, step, c.stream_id, c.seed_lo, c.seed_hi, w);
  const bool odd = (j & 1) != 0;
  box_muller(odd ? w[2] : w[0], odd ? w[3] : w[1], g[0], g[1]);
}

template <>
__device__ __forceinline__ void step_gaussians<6>(const Cfg& c, uint32_t step, int k, int j, float* g) {
  // pairs 3j, 3j+1, 3j+2 span blocks b0 = 3j/2 and b0 + 1
  const int q0 = 3 * j;
  const int b0 = q0 >> 1;
  uint32_t w[4], v[4];
  philox((uint32_t)b0, (uint32_t)k, step, c.stream_id, c.seed_lo, c.seed_hi, w);
  philox((uint32_t)(b0 + 1), (uint32_t)k, step, c.stream_id, c.seed_lo, c.seed_hi, v);
  // even q0: (b0,h0) (b0,h1) (b0+1,h0); odd q0: (b0,h1) (b0+1,h0) (b0+1,h1)
  const bool ev = (q0 & 1) == 0;
  box_muller(ev ? w[0] : w[2], ev ? w[1] : w[3], g[0], g[1]);
  box_muller(ev ? w[2] : v[0], ev ? w[3] : v[1], g[2], g[3]);
  box_muller(ev ? v[0] : v[2], ev ? v[1] : v[3], g[4], g[5]);
}

// ---------------------------------------------------------------------------
// Segmented wave primitives on DPP lane moves (segments of SEG = 32 or 64
// lanes; every lane participates).  GFX9 DPP: row_shr:n shifts within a row
// of 16 lanes, row_bcast:15 / row_bcast:31 feed a row's last lane into the
// next row(s), wave_shr:1 shifts the whole wave by one lane.
__device__ __forceinline__ float dpp_shr_row(float v, int n) {
  // bound_ctrl: lanes whose source is outside the row read 0
  switch (n) {
    case 1: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
    case 2: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));
    case 4: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));
    default: return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));
  }
}

template <int SEG>
__device__ __forceinline__ float seg_incl_scan(float v, int /*j*/) {
  v += dpp_shr_row(v, 1);
  v += dpp_shr_row(v, 2);
  v += dpp_shr_row(v, 4);
  v += dpp_shr_row(v, 8);
  // rows 1 and 3 add the total of rows 0 and 2
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xa, 0xf, false));
  if (SEG == 64) {
    // rows 2 and 3 add the total of rows 0-1
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xc, 0xf, false));
  }
  return v;
}

template <int SEG>
__device__ __forceinline__ float seg_excl_scan(float v, int j) {
  const float inc = seg_incl_scan<SEG>(v, j);
  const float t = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(inc), 0x138, 0xf, 0xf, true));
  return j == 0 ? 0.0f : t;
}

// value of lane `src` of this lane's segment (src < SEG, uniform across the
// wave); for SEG == 32 the two segments read their own lane
template <int SEG>
__device__ __forceinline__ float seg_bcast(float v, int src) {
  // readlane takes a wave-uniform lane index
  if (SEG == 64) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src + 32));
  return (__lane_id() < 32) ? a : b;
}
template <int SEG>
__device__ __forceinline__ int seg_bcast_i(int v, int src) {
  if (SEG == 64) return __builtin_amdgcn_readlane(v, src);
  const int a = __builtin_amdgcn_readlane(v, src);
  const int b = __builtin_amdgcn_readlane(v, src + 32);
  return (__lane_id() < 32) ? a : b;
}

// value of lane src0 (segment 0) / src1 (segment 1), both wave-uniform
template <int SEG>
__device__ __forceinline__ float seg_pick(float v, int src0, int src1) {
  if (SEG == 64) return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src0));
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src0));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32 + src1));
  return (__lane_id() < 32) ? a : b;
}
template <int SEG>
__device__ __forceinline__ int seg_pick_i(int v, int src0, int src1) {
  if (SEG == 64) return __builtin_amdgcn_readlane(v, src0);
  const int a = __builtin_amdgcn_readlane(v, src0);
  const int b = __builtin_amdgcn_readlane(v, 32 + src1);
  return (__lane_id() < 32) ? a : b;
}

// segment sum = last lane of the inclusive scan (fixed order: every lane of
// the segment receives the bitwise same value)
template <int SEG>
__device__ __forceinline__ float seg_sum(float v) {
  return seg_bcast<SEG>(seg_incl_scan<SEG>(v, 0), SEG - 1);
}

__device__ __forceinline__ float sq(float x) { return x * x; }

// squared distance with a fixed operation order, shared by every decision
// that compares a distance to a radius: d_i = a_i - b_i,
// s = fma(d_{p-1}, d_{p-1}, ... fma(d_1, d_1, d_0 * d_0))
__device__ __forceinline__ float dist2_2(float ax, float ay, float bx, float by) {
  const float dx = ax - bx, dy = ay - by;
  return __builtin_fmaf(dy, dy, dx * dx);
}
__device__ __forceinline__ float dist2_3(float ax, float ay, float az, float bx, float by, float bz) {
  const float dx = ax - bx, dy = ay - by, dz = az - bz;
  return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// agent-scope atomics for data shared between workgroups inside one kernel
__device__ __forceinline__ int ld_acquire(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// block-wide (blockDim.x == NT) exclusive scan of one int per thread;
// returns the exclusive prefix and writes the total.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int v, int* total) {
  __shared__ int s_w[NT / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = __shfl_up(inc, (unsigned)d, kWave);
    if (lane >= d) inc += t;
  }
  if (lane == kWave - 1) s_w[w] = inc;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) {
    if (i < w) base += s_w[i];
    tot += s_w[i];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

// block-wide (blockDim.x == NT) exclusive max-scan of one int per thread
// (identity -1); returns the maximum over the lower threads and writes the
// block maximum.
template <int NT>
__device__ __forceinline__ int block_excl_max(int v, int* total) {
  __shared__ int s_w[NT / kWave];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int t = __shfl_up(inc, (unsigned)d, kWave);
    if (lane >= d) inc = max(inc, t);
  }
  const int below = __shfl_up(inc, 1u, kWave);
  if (lane == kWave - 1) s_w[w] = inc;
  __syncthreads();
  int base = -1, tot = -1;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) {
    if (i < w) base = max(base, s_w[i]);
    tot = max(tot, s_w[i]);
  }
  __syncthreads();
  *total = tot;
  return lane > 0 ? max(base, below) : base;
}

}  // namespace cemppi
