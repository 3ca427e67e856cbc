// cluster.hip -- everything after the rollouts: pruning and stable compaction
// of the feasible set with the features of Eq. (12)-(13), DBSCAN
// (Sec. II-B.2), cluster statistics and selection (Alg. 1 [Cluster stats] /
// [Selection], Eq. (14)-(18)) and the path-integral update with the shift
// (Eq. (6)-(7), Eq. (19)-(20), Alg. 1 [Execute]).
//
// No block of a kernel waits for another.  Blocks combine results only
// through integer atomics whose outcome does not depend on their order
// (neighbour counts, minima, bit ORs); every floating-point reduction that
// several blocks need is recomputed by each of them from the previous
// kernel's outputs in a fixed order (so results are deterministic), and the
// work that needs a single view runs in a one-block kernel.
//
// DBSCAN plan (exact, deterministic; V = number of feasible rollouts):
//  1. count   tiled all-pairs eps-neighbour count -> core flags
//  2. mcn     tiled all-pairs lowest-index core neighbour; for a core point it
//             is its hook target, for a non-core point it is exactly the
//             border rule (join the cluster of the lowest-index core neighbour)
//  3. roots   a core point with no core neighbour of lower index roots a
//             tree (flag words from step 2); trees are numbered by root index
//  4. trees   tiled pass over core-core neighbour pairs of different trees;
//             each block first follows the hooks of its points (indices
//             strictly decrease) to their roots, then ORs the tree
//             adjacency bits it saw into the 64 rows of the tree graph
//  5. tree CC connected components of the (small) tree graph; the cluster of
//             a component is ranked by its lowest root index, which is the
//             lowest core index of the cluster
// With more than 64 trees, steps 4-5 are replaced by an exact
// single-workgroup union-find over the core graph.
// A single planner of at most kAdjMaxK rollouts runs steps 1, 2 and 4 on an
// eps-adjacency bitmap instead (1b, 2b, 4b below): one tiled pass evaluates
// each pair once and stores the outcome, the other two read bits.
#include "device.hpp"
#include "launch.hpp"

namespace cemppi {

template <int P>
struct ZVec;
// Morton cell of a feature (points of the unit disc / ball; values outside
// [-1, 1] are clamped): 64 x 64 cells in 2-D, 16 x 16 x 16 in 3-D, 12 bits.
__device__ __forceinline__ int morton_q(float v, int g) {
  const int q = (int)floorf((v + 1.f) * (0.5f * (float)g));
  return q < 0 ? 0 : (q >= g ? g - 1 : q);
}
__device__ __forceinline__ unsigned spread2(unsigned v) {  // 6 bits -> every 2nd bit
  v = (v | (v << 4)) & 0x0F0Fu;
  v = (v | (v << 2)) & 0x3333u;
  v = (v | (v << 1)) & 0x5555u;
  return v;
}
__device__ __forceinline__ unsigned spread3(unsigned v) {  // 4 bits -> every 3rd bit
  v = (v | (v << 4)) & 0x0C3u;
  v = (v | (v << 2)) & 0x249u;
  return v;
}
template <>
struct ZVec<2> {
  using T = float2;
  static __device__ __forceinline__ T far() { return make_float2(1e30f, 1e30f); }
  static __device__ __forceinline__ T nfar() { return make_float2(-1e30f, -1e30f); }
  static __device__ __forceinline__ float d2(T a, T b) { return dist2_2(a.x, a.y, b.x, b.y); }
  static __device__ __forceinline__ int key(T a) {
    return (int)(spread2((unsigned)morton_q(a.x, 64)) | (spread2((unsigned)morton_q(a.y, 64)) << 1));
  }
  static __device__ __forceinline__ float4 lift(T a) { return make_float4(a.x, a.y, 0.f, 0.f); }
};
template <>
struct ZVec<3> {
  using T = float4;
  static __device__ __forceinline__ T far() { return make_float4(1e30f, 1e30f, 1e30f, 0.f); }
  static __device__ __forceinline__ T nfar() { return make_float4(-1e30f, -1e30f, -1e30f, 0.f); }
  static __device__ __forceinline__ float d2(T a, T b) { return dist2_3(a.x, a.y, a.z, b.x, b.y, b.z); }
  static __device__ __forceinline__ int key(T a) {
    return (int)(spread3((unsigned)morton_q(a.x, 16)) | (spread3((unsigned)morton_q(a.y, 16)) << 1) |
                 (spread3((unsigned)morton_q(a.z, 16)) << 2));
  }
  static __device__ __forceinline__ float4 lift(T a) { return make_float4(a.x, a.y, a.z, 0.f); }
};

// Lower bound of the squared distance between two points of two boxes.
__device__ __forceinline__ float box_gap2(float4 alo, float4 ahi, float4 blo, float4 bhi) {
  const float gx = fmaxf(0.f, fmaxf(blo.x - ahi.x, alo.x - bhi.x));
  const float gy = fmaxf(0.f, fmaxf(blo.y - ahi.y, alo.y - bhi.y));
  const float gz = fmaxf(0.f, fmaxf(blo.z - ahi.z, alo.z - bhi.z));
  return gx * gx + gy * gy + gz * gz;
}
// Tile pairs whose boxes are farther apart than eps hold no neighbour pair;
// the margin is far above the FP32 rounding of the pair distances.
__device__ __forceinline__ bool tiles_apart(const Cfg& c, const Bufs& b, int I, int J) {
  return box_gap2(b.tlo[I], b.thi[I], b.tlo[J], b.thi[J]) > c.eps2 * (1.f + 1e-4f) + 1e-12f;
}

__device__ __forceinline__ bool is_min_field(int f) { return f == P_SMIN_ALL || f == P_SMIN_FEAS; }

// ---------------------------------------------------------------------------
// Reduction of the rollout-group partial records (256-thread blocks):
// thread t owns records t, t+256, ... (coalesced), each wave combines its
// lanes by an xor butterfly (every lane ends with the same value), and the
// four wave results are added in wave order.  Also returns the number of
// feasible rollouts in records [0, upto).  A thread requests kRecBatch of its
// records before adding any of them (in the same order).
__device__ void reduce_partials(const Cfg& c, const Bufs& b, int upto, float* s_tot, int* s_before) {
  __shared__ float s_w[4][kPart + 1];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
  float acc[kPart + 1];
#pragma unroll
  for (int f = 0; f < kPart; ++f) acc[f] = is_min_field(f) ? INFINITY : 0.f;
  acc[kPart] = 0.f;
  const float4* rows = reinterpret_cast<const float4*>(b.part);
  for (int i0 = tid; i0 < c.npart; i0 += 256 * kRecBatch) {
    float4 x[kRecBatch], y[kRecBatch], z[kRecBatch];
#pragma unroll
    for (int r = 0; r < kRecBatch; ++r) {
      const int i = i0 + r * 256;
      if (i < c.npart) {
        x[r] = rows[3 * i];
        y[r] = rows[3 * i + 1];
        z[r] = rows[3 * i + 2];
      }
    }
#pragma unroll
    for (int r = 0; r < kRecBatch; ++r) {
      const int i = i0 + r * 256;
      if (i >= c.npart) break;
      const float v[kPart] = {x[r].x, x[r].y, x[r].z, x[r].w, y[r].x, y[r].y,
                              y[r].z, y[r].w, z[r].x, z[r].y, z[r].z, z[r].w};
#pragma unroll
      for (int f = 0; f < kPart; ++f) acc[f] = is_min_field(f) ? fminf(acc[f], v[f]) : acc[f] + v[f];
      if (i < upto) acc[kPart] += v[P_NFEAS];
    }
  }
#pragma unroll
  for (int f = 0; f <= kPart; ++f) {
    float v = acc[f];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float o = __shfl_xor(v, off, kWave);
      v = (f < kPart && is_min_field(f)) ? fminf(v, o) : v + o;
    }
    acc[f] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f <= kPart; ++f) s_w[wv][f] = acc[f];
  }
  __syncthreads();
  if (tid <= kPart) {
    const bool mn = tid < kPart && is_min_field(tid);
    const float a = s_w[0][tid], b1 = s_w[1][tid], b2 = s_w[2][tid], b3 = s_w[3][tid];
    const float t = mn ? fminf(fminf(fminf(a, b1), b2), b3) : ((a + b1) + b2) + b3;
    if (tid < kPart) s_tot[tid] = t;
    else *s_before = (int)t;
  }
  __syncthreads();
}

// Branch of Alg. 1 and the reference point of Eq. (11) from the totals.
struct Totals {
  int branch, ncol, nfeas, nref;
  uint32_t status;
  float ref[3];
};
__device__ __forceinline__ Totals decide(const Cfg& c, const float* tot, int bad) {
  Totals t;
  t.ncol = (int)tot[P_NCOL];
  t.nfeas = (int)tot[P_NFEAS];
  const int na = (int)tot[P_NREF];
  if (bad) {
    t.branch = 1;
    t.status = 16u;
  } else if (t.ncol == 0) {
    t.branch = 1;
    t.status = 1u;
  } else if (t.nfeas == 0) {
    t.branch = 2;
    t.status = 2u;
  } else {
    t.branch = 0;
    t.status = 0u;
  }
  // the rollouts whose first contact is o*, or every colliding rollout
  const bool useA = na > 0;
  const float cnt = useA ? (float)na : (float)t.ncol;
  for (int i = 0; i < 3; ++i) {
    const float sum = useA ? tot[P_SUM_REF + i] : tot[P_SUM_COL + i];
    t.ref[i] = (t.branch == 0 && i < c.p) ? sum / cnt : 0.f;
  }
  t.nref = t.branch == 0 ? (useA ? na : t.ncol) : 0;
  return t;
}

// ---------------------------------------------------------------------------
// Pruning (Eq. (9)-(10)), reference point (Eq. (11)), stable compaction of V
// in ascending rollout order, features z (Eq. (13)) and the DBSCAN arrays.
// Block 0 publishes the totals.
// ---------------------------------------------------------------------------
// Angular buckets of the windowed DBSCAN (k_wdbscan below).  The
// bucket coordinate of a feature is its angle mapped to [0, kWinBins]; a
// ring point has a squared norm within [w_r2lo, w_r2hi]; every other point
// goes to the extra bucket kWinBins ("off the ring").
__device__ __forceinline__ float win_u(const Cfg& c, float2 z) {
  return fmaxf(0.f, (atan2f(z.y, z.x) + 3.14159265f) * c.w_scale);
}
__device__ __forceinline__ int win_bucket(float u) { return min((int)u, kWinBins - 1); }
__device__ __forceinline__ bool win_ring(const Cfg& c, float2 z) {
  const float n2 = __builtin_fmaf(z.y, z.y, z.x * z.x);
  return n2 >= c.w_r2lo && n2 <= c.w_r2hi;
}
// bucket and slot of point `rank`: the slot is its arrival order in the
// bucket (any order serves: no result depends on the order inside a bucket)
__device__ __forceinline__ void win_bin(const Cfg& c, const Bufs& b, float2 zz, int rank) {
  const int bkt = win_ring(c, zz) ? win_bucket(win_u(c, zz)) : kWinBins;
  const int slot = atomicAdd(&b.wcnt[bkt], 1);
  b.wkey[rank] = (bkt << kWinShift) | slot;
}
__device__ __forceinline__ void win_bin(const Cfg&, const Bufs&, float4, int) {}

template <int P, bool BIN = false>
__device__ __forceinline__ void compact_body(const Cfg& c, const Bufs& b, int bx, int by, int nbx) {
  using ZT = typename ZVec<P>::T;
  __shared__ float s_tot[kPart + 1];
  __shared__ int s_before;
  // the rollout's own record and the input flag are requested before the
  // partials (they are only needed on the clustering branch)
  // (unconditional loads at a clamped index keep them out of branches)
  const int k = bx * 256 + threadIdx.x;
  const bool ink = k < c.K;
  const int kc = ink ? k : c.K - 1;
  const int bad = b.ctrl->nonfinite;
  const int colk = b.col[kc];
  const float Sk = b.S[kc];
  float pk[3] = {0.f, 0.f, 0.f}, gk[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < P; ++i) {
    pk[i] = b.pT[(size_t)kc * P + i];
    gk[i] = b.g[(size_t)kc * P + i];
  }
  const int blk0 = (bx * 256) / kGroup;
  reduce_partials(c, b, blk0, s_tot, &s_before);
  const Totals T = decide(c, s_tot, bad);
  if (bx == 0 && threadIdx.x == 0) {
    Ctrl* ct = b.ctrl;
    ct->n_col = T.ncol;
    ct->n_feas = T.nfeas;
    ct->n_ref = T.nref;
    ct->branch = T.branch;
    ct->status = T.status;
    ct->smin_all = s_tot[P_SMIN_ALL];
    ct->smin_feas = s_tot[P_SMIN_FEAS];
    ct->M = 0;
    ct->sel = -1;
    for (int i = 0; i < 3; ++i) ct->ref[i] = T.ref[i];
    // Eq. (17) for o*, once per replan on the clustering branch (the
    // selection reads it): the mean of H'-1 finite differences telescopes
    // to (o_t - o_{t-H'+1}) / ((H'-1) dt)
    float v[3] = {0.f, 0.f, 0.f};
    int Hp = 0;
    if (c.scene_mode == 1 && T.branch == 0) {
      const int hc = ct->hist_count;
      Hp = hc < c.H ? hc : c.H;
      const int o = ct->closest;
      if (Hp >= 2 && o >= 0) {
        const int h0 = ct->hist_head;
        const int h1 = (h0 - (Hp - 1) + 2 * c.H) % c.H;
        const float* pa = b.hist + ((size_t)h0 * c.max_obs + o) * c.p;
        const float* pz = b.hist + ((size_t)h1 * c.max_obs + o) * c.p;
        const float den = (float)(Hp - 1) * c.dt;
        v[0] = (pa[0] - pz[0]) / den;
        v[1] = (pa[1] - pz[1]) / den;
        if (c.p == 3) v[2] = (pa[2] - pz[2]) / den;
      }
    }
    const float nv = sqrtf(__builtin_fmaf(v[2], v[2], __builtin_fmaf(v[1], v[1], v[0] * v[0])));
    for (int i = 0; i < 3; ++i) {
      ct->v_obs[i] = v[i];
      ct->v_hat[i] = v[i] / (nv + c.norm_eps);
    }
    ct->dyn_h = Hp;
    ct->dyn_ok = (c.scene_mode == 1 && Hp >= 2 && !(nv < c.v_obs_min)) ? 1 : 0;
  }
  if (T.branch != 0) return;
  const int feas = ink ? !colk : 0;
  int tot;
  const int local = block_excl_scan<256>(feas, &tot);
  if (!feas) return;
  const int rank = s_before + local;
  float d[3] = {0.f, 0.f, 0.f}, g[3] = {0.f, 0.f, 0.f};
  for (int i = 0; i < P; ++i) {
    d[i] = pk[i] - T.ref[i];
    g[i] = gk[i];
  }
  const float nd = sqrtf(__builtin_fmaf(d[2], d[2], __builtin_fmaf(d[1], d[1], d[0] * d[0])));
  const float den = nd + c.norm_eps;
  ZT zz, gg;
  if constexpr (P == 2) {
    zz = make_float2(d[0] / den, d[1] / den);
    gg = make_float2(g[0], g[1]);
  } else {
    zz = make_float4(d[0] / den, d[1] / den, d[2] / den, 0.f);
    gg = make_float4(g[0], g[1], g[2], 0.f);
  }
  reinterpret_cast<ZT*>(b.z)[rank] = zz;
  if constexpr (BIN) win_bin(c, b, zz, rank);
  reinterpret_cast<ZT*>(b.gv)[rank] = gg;
  b.vidx[rank] = k;
  b.Sv[rank] = Sk;
  b.ncount[rank] = 0;
  b.mcn[rank] = kInt32Max;
  b.root[rank] = -1;
  b.label[rank] = -1;
  if ((rank & 63) == 0) b.hookmask[rank >> 6] = 0ull;
  if (rank < kMaxTrees) b.tadj[rank] = 0ull;  // rows of trees 0 .. min(V, 64) - 1
}

template <int P, bool BIN>
__global__ __launch_bounds__(256) void k_compact(Cfg c, Bufs b) {
  compact_body<P, BIN>(c, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x);
}

// per-point DBSCAN state for a stage call on caller features
__global__ void k_init_points(Bufs b, int V) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= V) return;
  b.ncount[a] = 0;
  b.mcn[a] = kInt32Max;
  b.root[a] = -1;
  b.label[a] = -1;
  if ((a & 63) == 0) b.hookmask[a >> 6] = 0ull;
  if (a < kMaxTrees) b.tadj[a] = 0ull;
}

// number of points DBSCAN runs on: caller features (stage) or the feasible set
__device__ __forceinline__ int dbscan_V(const Bufs& b, const float* zin, int Vin) {
  return zin ? Vin : (b.ctrl->branch == 0 ? b.ctrl->n_feas : 0);
}

// Tiled passes: block (g, I) takes row tile I against the column tiles
// g*kColGroup .. g*kColGroup + kColGroup - 1 (clipped to the tiles in use),
// the row point in registers and each column tile staged through LDS.
__device__ __forceinline__ int ntiles_of(int V) { return (V + kTile - 1) / kTile; }

// 0. spatial order (batched form): the features sorted by Morton cell
// (counting sort in one block per planner), with their original indices, and
// the bounding box of every tile of kTile consecutive sorted points.  The
// batched count and tree-adjacency passes work on this order and skip tile
// pairs whose boxes are farther apart than eps; every rule that names a point
// (lowest-index core neighbour, roots, labels) uses the original index, so
// no result depends on the order.  The single-planner path keeps the
// original order: at one planner's sizes the extra launch costs more than
// the culling saves.
template <int P>
__device__ __forceinline__ void sort_body(const Cfg& c, const Bufs& b, const float* zin, int Vin) {
  using ZT = typename ZVec<P>::T;
  __shared__ int s_bin[kSortBins];
  const int V = dbscan_V(b, zin, Vin);
  if (V == 0) return;
  const ZT* z = reinterpret_cast<const ZT*>(zin ? zin : b.z);
  ZT* zs = reinterpret_cast<ZT*>(b.zs);
  const int tid = threadIdx.x;
  for (int i = tid; i < kSortBins; i += kFinThreads) s_bin[i] = 0;
  __syncthreads();
  for (int a = tid; a < V; a += kFinThreads) atomicAdd(&s_bin[ZVec<P>::key(z[a])], 1);
  __syncthreads();
  constexpr int PER = kSortBins / kFinThreads;
  int loc[PER], sum = 0;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    loc[q] = s_bin[tid * PER + q];
    sum += loc[q];
  }
  int tot;
  int off = block_excl_scan<kFinThreads>(sum, &tot);
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    s_bin[tid * PER + q] = off;
    off += loc[q];
  }
  __syncthreads();
  for (int a = tid; a < V; a += kFinThreads) {
    const ZT v = z[a];
    const int pos = atomicAdd(&s_bin[ZVec<P>::key(v)], 1);
    zs[pos] = v;
    b.sid[pos] = a;
  }
  __syncthreads();
  // tile boxes: wave w takes tiles w, w + 16, ...; two points per lane
  const int lane = tid & (kWave - 1), w = tid / kWave;
  const int nt = ntiles_of(V);
  for (int t = w; t < nt; t += kFinThreads / kWave) {
    float4 lo = make_float4(INFINITY, INFINITY, INFINITY, 0.f), hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.f);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int k = t * kTile + h * kWave + lane;
      if (k < V) {
        const float4 v = ZVec<P>::lift(zs[k]);
        lo = make_float4(fminf(lo.x, v.x), fminf(lo.y, v.y), fminf(lo.z, v.z), 0.f);
        hi = make_float4(fmaxf(hi.x, v.x), fmaxf(hi.y, v.y), fmaxf(hi.z, v.z), 0.f);
      }
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
      lo.x = fminf(lo.x, __shfl_xor(lo.x, d, kWave));
      lo.y = fminf(lo.y, __shfl_xor(lo.y, d, kWave));
      lo.z = fminf(lo.z, __shfl_xor(lo.z, d, kWave));
      hi.x = fmaxf(hi.x, __shfl_xor(hi.x, d, kWave));
      hi.y = fmaxf(hi.y, __shfl_xor(hi.y, d, kWave));
      hi.z = fmaxf(hi.z, __shfl_xor(hi.z, d, kWave));
    }
    if (lane == 0) {
      b.tlo[t] = lo;
      b.thi[t] = hi;
    }
  }
}

// AND of a predicate over the NT threads of a block (a barrier for all of
// them).  Each wave posts whether any of its lanes is false; consecutive
// calls must be separated by another barrier of the block (the tiled passes
// stage a tile between calls), so one word per wave suffices.  (The
// library's block-wide AND reads the block size from the dispatch packet,
// one more memory round trip per kernel.)
template <int NT>
__device__ __forceinline__ bool block_and(bool p, int* s_w) {
  const unsigned long long f = __ballot(!p);
  if ((threadIdx.x & (kWave - 1)) == 0) s_w[threadIdx.x / kWave] = f != 0ull ? 1 : 0;
  __syncthreads();
  int any = 0;
#pragma unroll
  for (int i = 0; i < NT / kWave; ++i) any |= s_w[i];
  return any == 0;
}

// 1. neighbour counts: for each row point, its neighbours among the block's
// column points (closed ball, itself included), in sorted order.  With CS > 1,
// CS threads share a row (thread = row + kTile * split), each taking 1/CS of
// every column tile: more waves for the latency of the LDS loop when the
// feasible set is small.
template <int P, int COLG = kColGroup, bool SORTED = false, int CS = 1>
__device__ __forceinline__ void count_body(const Cfg& c, const Bufs& b, int bx, int by, int nbx,
                                           const float* __restrict__ zin, int Vin) {
  using ZT = typename ZVec<P>::T;
  constexpr int NT = kTile * CS, SPAN = kTile / CS;
  __shared__ int s_all[NT / kWave];
  __shared__ ZT s_z[kTile];
  __shared__ int s_part[CS][kTile];
  const int r = CS > 1 ? (int)(threadIdx.x & (kTile - 1)) : (int)threadIdx.x;
  const int q = CS > 1 ? (int)(threadIdx.x / kTile) : 0;
  const int V = dbscan_V(b, zin, Vin);
  const int nt = ntiles_of(V);
  const int I = by, J0 = bx * COLG;
  if (I >= nt || J0 >= nt) return;
  const int J1 = min(J0 + COLG, nt);
  if constexpr (SORTED) {
    // a block whose column tiles are all apart from the row tile has no pair
    bool any = false;
    for (int J = J0; J < J1; ++J) any |= !tiles_apart(c, b, I, J);
    if (!any) return;
  }
  const ZT* z = reinterpret_cast<const ZT*>(SORTED ? b.zs : (zin ? zin : b.z));
  const int k = I * kTile + r;
  const ZT zk = k < V ? z[k] : ZVec<P>::far();
  const int ok_k = SORTED ? (k < V ? b.sid[k] : 0) : k;
  ZT zl[COLG];
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int l = (J0 + u) * kTile + r;
    zl[u] = (q == 0 && J0 + u < J1 && l < V) ? z[l] : ZVec<P>::far();
  }
  const float r2 = c.eps2;
  int cnt = 0;  // this split's count
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int J = J0 + u;
    if (J >= J1) break;
    if (SORTED && tiles_apart(c, b, I, J)) continue;
    // only the core test needs the count: once every row of the block has
    // minPts neighbours in this chunk, the rest of the chunk cannot change it
    int tot = cnt;
    if constexpr (CS > 1) {
      s_part[q][r] = cnt;
      __syncthreads();
      tot = 0;
#pragma unroll
      for (int i = 0; i < CS; ++i) tot += s_part[i][r];
    }
    if (block_and<NT>(k >= V || tot >= c.min_pts, s_all)) break;
    if (q == 0) s_z[r] = zl[u];
    __syncthreads();
    const int ncol = min(kTile, V - J * kTile);
    const int t1 = CS > 1 ? min(ncol, (q + 1) * SPAN) : ncol;
    for (int t = q * SPAN; t < t1; ++t) cnt += ZVec<P>::d2(zk, s_z[t]) <= r2 ? 1 : 0;
  }
  if constexpr (CS > 1) {
    s_part[q][r] = cnt;
    __syncthreads();
    if (q == 0) {
      cnt = 0;
#pragma unroll
      for (int i = 0; i < CS; ++i) cnt += s_part[i][r];
    }
  }
  if (q == 0 && k < V && cnt) atomicAdd(&b.ncount[ok_k], cnt);
}

template <int P, int CS>
__global__ __launch_bounds__(kTile * CS) void k_count(Cfg c, Bufs b, const float* __restrict__ zin, int Vin) {
  count_body<P, kCntGroup, false, CS>(c, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, zin, Vin);
}

// 2. lowest-index core neighbour of every point (core points include
// themselves).  This pass runs in the original order: column tiles ascend,
// so the first hit of a row is its minimum within the block, and a block
// stops once every row has one (in dense regions after the first tile).
// The block whose columns hold the row tile also writes the tile's core
// flags (one 64-bit word per wave), and every block flags the rows that have
// a core neighbour of lower index: a core point without one is the root of
// its hook tree.
template <int P, int COLG = kColGroup, int CS = 1>
__device__ __forceinline__ void mcn_body(const Cfg& c, const Bufs& b, int bx, int by, int nbx,
                                         const float* __restrict__ zin, int Vin) {
  using ZT = typename ZVec<P>::T;
  constexpr int NT = kTile * CS, SPAN = kTile / CS;
  __shared__ int s_all[NT / kWave];
  __shared__ ZT s_z[kTile];
  __shared__ int s_part[CS][kTile];
  // CS threads share a row as in the count pass; the row's hit is the
  // lowest of its splits' first hits
  const int r = CS > 1 ? (int)(threadIdx.x & (kTile - 1)) : (int)threadIdx.x;
  const int q = CS > 1 ? (int)(threadIdx.x / kTile) : 0;
  const int V = dbscan_V(b, zin, Vin);
  const int nt = ntiles_of(V);
  const int I = by, J0 = bx * COLG;
  if (I >= nt || J0 >= nt) return;
  const int J1 = min(J0 + COLG, nt);
  const ZT* z = reinterpret_cast<const ZT*>(zin ? zin : b.z);
  const int k = I * kTile + r;
  const ZT zk = k < V ? z[k] : ZVec<P>::far();
  const bool diag = J0 <= I && I < J1;
  const int nck = (q == 0 && diag && k < V) ? b.ncount[k] : 0;
  ZT zl[COLG];
  int ncl[COLG];
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int l = (J0 + u) * kTile + r;
    const bool ok = q == 0 && J0 + u < J1 && l < V;
    zl[u] = ok ? z[l] : ZVec<P>::far();
    ncl[u] = ok ? b.ncount[l] : 0;
  }
  if (diag && q == 0) {
    const unsigned long long cm = __ballot(k < V && nck >= c.min_pts);
    if ((threadIdx.x & (kWave - 1)) == 0 && k < V) b.coremask[k >> 6] = cm;
  }
  const float r2 = c.eps2;
  int m = kInt32Max;  // this split's first hit
  // lowest hit of the row over its splits (a barrier when CS > 1: every
  // thread calls it)
  auto row_min = [&]() {
    int mm = m;
    if constexpr (CS > 1) {
      s_part[q][r] = m;
      __syncthreads();
#pragma unroll
      for (int i = 0; i < CS; ++i) mm = min(mm, s_part[i][r]);
    }
    return mm;
  };
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int J = J0 + u;
    if (J >= J1) break;
    const int mm = row_min();
    if (block_and<NT>(k >= V || mm != kInt32Max, s_all)) break;
    // non-core columns are parked far away: they can never be a neighbour here
    if (q == 0) s_z[r] = ncl[u] >= c.min_pts ? zl[u] : ZVec<P>::far();
    __syncthreads();
    if (m == kInt32Max) {
      const int ncol = min(kTile, V - J * kTile);
      const int t1 = CS > 1 ? min(ncol, (q + 1) * SPAN) : ncol;
      for (int t = q * SPAN; t < t1; ++t) {
        const bool h = ZVec<P>::d2(zk, s_z[t]) <= r2;
        m = (h && m == kInt32Max) ? J * kTile + t : m;
      }
    }
  }
  m = row_min();
  if (q == 0) {
    if (k < V && m != kInt32Max) atomicMin(&b.mcn[k], m);
    const unsigned long long hk = __ballot(k < V && m < k);
    if (hk && (threadIdx.x & (kWave - 1)) == 0) atomicOr(&b.hookmask[k >> 6], hk);
  }
}

template <int P, int CS>
__global__ __launch_bounds__(kTile * CS) void k_mcn(Cfg c, Bufs b, const float* __restrict__ zin, int Vin) {
  mcn_body<P, kCntGroup, CS>(c, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, zin, Vin);
}

// 3. roots of the hook forest: each core point hooks to its lowest-index core
// neighbour, so indices decrease along a chain and the walk ends at a point
// that hooks to itself.  The chains of one thread advance together, all
// their loads in flight at once.
template <int NR>
__device__ __forceinline__ void follow_roots(const int* __restrict__ mcn, int (&r)[NR]) {
  while (true) {
    int nx[NR];
#pragma unroll
    for (int u = 0; u < NR; ++u) nx[u] = r[u] >= 0 ? mcn[r[u]] : r[u];
    bool more = false;
#pragma unroll
    for (int u = 0; u < NR; ++u) {
      more |= nx[u] != r[u];
      r[u] = nx[u];
    }
    if (!more) break;
  }
}

// Tree numbering: exclusive prefix of root counts over the root-flag words
// (core and not hooked to a lower index), computed by each block that needs
// it into LDS (the flag words are kept in LDS too); returns the number of
// trees.
template <int NT>
__device__ int tree_prefix(const Bufs& b, int V, int* s_woff, unsigned long long* s_rm) {
  const int nwords = (V + 63) >> 6;
  const int per = (nwords + NT - 1) / NT;
  const int lo = min((int)threadIdx.x * per, nwords), hi = min(lo + per, nwords);
  int mine = 0;
  for (int i = lo; i < hi; ++i) {
    const unsigned long long m = b.coremask[i] & ~b.hookmask[i];
    s_rm[i] = m;
    mine += __popcll(m);
  }
  int tot;
  int off = block_excl_scan<NT>(mine, &tot);
  for (int i = lo; i < hi; ++i) {
    s_woff[i] = off;
    off += __popcll(s_rm[i]);
  }
  __syncthreads();
  return tot;
}

// The same numbering in two steps, so that a kernel can request the flag
// words together with its other operands: root_words loads this thread's
// words (the partition of tree_prefix, at most PER words), tree_prefix_of
// numbers them.
template <int NT, int PER>
__device__ __forceinline__ void root_words(const Bufs& b, int V, unsigned long long (&w)[PER], int& lo,
                                           int& hi) {
  const int nwords = (V + 63) >> 6;
  const int per = (nwords + NT - 1) / NT;
  lo = min((int)threadIdx.x * per, nwords);
  hi = min(lo + per, nwords);
#pragma unroll
  for (int i = 0; i < PER; ++i) w[i] = lo + i < hi ? (b.coremask[lo + i] & ~b.hookmask[lo + i]) : 0ull;
}

template <int NT, int PER>
__device__ int tree_prefix_of(const unsigned long long (&w)[PER], int lo, int hi, int* s_woff,
                              unsigned long long* s_rm) {
  int mine = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (lo + i < hi) {
      s_rm[lo + i] = w[i];
      mine += __popcll(w[i]);
    }
  int tot;
  int off = block_excl_scan<NT>(mine, &tot);
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (lo + i < hi) {
      s_woff[lo + i] = off;
      off += __popcll(w[i]);
    }
  __syncthreads();
  return tot;
}

__device__ __forceinline__ int tree_id(const unsigned long long* s_rm, const int* s_woff, int r) {
  const int w = r >> 6, bit = r & 63;
  const unsigned long long below = bit ? (s_rm[w] & ((1ull << bit) - 1ull)) : 0ull;
  return s_woff[w] + __popcll(below);
}

constexpr int kMaxWords = (65536 + 63) / 64;

// 4. tree adjacency over the upper triangle of tiles (J >= I; the closure
// makes the relation symmetric): for every core-core neighbour pair (row k,
// column l) of different trees set bit tree(l) in the row of tree(k).  Block
// (g, I) gathers its rows in LDS and ORs the nonzero ones into the global
// rows (an exact, order-independent reduction).
__device__ __forceinline__ bool adj_block_live(int I, int g, int nt) {
  const int J0 = g * kColGroup;
  return I < nt && J0 < nt && J0 + kColGroup > I;
}

template <int P, bool SORTED = false, int CS = 1>
__device__ __forceinline__ void tree_adj_body(const Cfg& c, const Bufs& b, int bx, int by, int nbx,
                                              const float* __restrict__ zin, int Vin) {
  using ZT = typename ZVec<P>::T;
  constexpr int NT = kTile * CS, SPAN = kTile / CS;
  // CS threads share a row as in the count pass; split 0 stages the columns
  const int r = CS > 1 ? (int)(threadIdx.x & (kTile - 1)) : (int)threadIdx.x;
  const int q = CS > 1 ? (int)(threadIdx.x / kTile) : 0;
  __shared__ ZT s_z[kTile];
  __shared__ uint2 s_bit[kTile];  // tree bit of the column point as two words, 0 if not core
  __shared__ int s_woff[kMaxWords];
  __shared__ unsigned long long s_rm[kMaxWords];
  __shared__ unsigned long long s_adj[kMaxTrees];
  const int V = dbscan_V(b, zin, Vin);
  const int nt = ntiles_of(V);
  const int I = by, g = bx;
  if (!adj_block_live(I, g, nt)) return;
  const ZT* z = reinterpret_cast<const ZT*>(SORTED ? b.zs : (zin ? zin : b.z));
  const int J0 = max(g * kColGroup, I), J1 = min(g * kColGroup + kColGroup, nt);
  if constexpr (SORTED) {
    bool any = false;
    for (int J = J0; J < J1; ++J) any |= !tiles_apart(c, b, I, J);
    if (!any) return;
  }
  // every operand of the block is requested before the first wait (sorted
  // positions first, then the per-point arrays at the original indices)
  const int k = I * kTile + r;
  const int idk = SORTED ? (k < V ? b.sid[k] : 0) : k;
  const ZT zk0 = k < V ? z[k] : ZVec<P>::far();
  int idl[kColGroup], ncl[kColGroup], rl[kColGroup];
  ZT zl[kColGroup];
#pragma unroll
  for (int u = 0; u < kColGroup; ++u) {
    const int l = (J0 + u) * kTile + r;
    const bool ok = q == 0 && J0 + u < J1 && l < V;
    idl[u] = ok ? (SORTED ? b.sid[l] : l) : -1;
    zl[u] = ok ? z[l] : ZVec<P>::far();
  }
  const int nck = k < V ? b.ncount[idk] : 0;
  const int hk = k < V ? b.mcn[idk] : -1;
#pragma unroll
  for (int u = 0; u < kColGroup; ++u) {
    ncl[u] = idl[u] >= 0 ? b.ncount[idl[u]] : 0;
    rl[u] = idl[u] >= 0 ? b.mcn[idl[u]] : -1;
  }
  // roots of the row point (slot 0) and the column points, -1 if not core
  int rt[kColGroup + 1];
  rt[0] = nck >= c.min_pts ? hk : -1;
#pragma unroll
  for (int u = 0; u < kColGroup; ++u) rt[u + 1] = ncl[u] >= c.min_pts ? rl[u] : -1;
  follow_roots(b.mcn, rt);
  const int rk = rt[0];
#pragma unroll
  for (int u = 0; u < kColGroup; ++u) rl[u] = rt[u + 1];
  // the block whose columns hold the row tile records the tile's roots for
  // the closure and the labels
  if (q == 0 && g * kColGroup <= I && I < g * kColGroup + kColGroup && k < V) b.root[idk] = rk;
  const int R = tree_prefix<NT>(b, V, s_woff, s_rm);
  if (R < 2 || R > kMaxTrees) return;
  if (threadIdx.x < kMaxTrees) s_adj[threadIdx.x] = 0ull;
  const int tk = nck >= c.min_pts ? tree_id(s_rm, s_woff, rk) : -1;
  const ZT zk = tk >= 0 ? zk0 : ZVec<P>::far();
  const float r2 = c.eps2;
  uint32_t mlo = 0u, mhi = 0u;
#pragma unroll
  for (int u = 0; u < kColGroup; ++u) {
    const int J = J0 + u;
    if (J >= J1) break;
    if (SORTED && tiles_apart(c, b, I, J)) continue;
    const int tl = ncl[u] >= c.min_pts ? tree_id(s_rm, s_woff, rl[u]) : -1;
    __syncthreads();
    if (q == 0) {
      s_z[r] = tl >= 0 ? zl[u] : ZVec<P>::far();
      s_bit[r] = tl < 0 ? make_uint2(0u, 0u)
                        : (tl < 32 ? make_uint2(1u << tl, 0u) : make_uint2(0u, 1u << (tl - 32)));
    }
    __syncthreads();
    if (tk >= 0) {
      // branch-free: both LDS words are read for every column
      const int ncol = min(kTile, V - J * kTile);
      const int t1 = CS > 1 ? min(ncol, (q + 1) * SPAN) : ncol;
#pragma unroll 8
      for (int t = q * SPAN; t < t1; ++t) {
        const uint2 bt = s_bit[t];
        const uint32_t h = ZVec<P>::d2(zk, s_z[t]) <= r2 ? 0xffffffffu : 0u;
        mlo |= bt.x & h;
        mhi |= bt.y & h;
      }
    }
  }
  if (tk >= 0) {
    unsigned long long mask = ((unsigned long long)mhi << 32) | mlo;
    mask &= ~(1ull << tk);
    if (mask) atomicOr(&s_adj[tk], mask);
  }
  __syncthreads();
  // OR is exact and commutative: the rows do not depend on the block order
  if (threadIdx.x < R && s_adj[threadIdx.x]) atomicOr(&b.tadj[threadIdx.x], s_adj[threadIdx.x]);
}

template <int P, int CS>
__global__ __launch_bounds__(kTile * CS) void k_tree_adj(Cfg c, Bufs b, const float* __restrict__ zin, int Vin) {
  tree_adj_body<P, false, CS>(c, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, zin, Vin);
}

// ---------------------------------------------------------------------------
// DBSCAN on the eps-adjacency bitmap (single planner, K <= kAdjMaxK).  The
// three distance passes above each evaluate about half of all pairs; here one
// tiled pass evaluates every pair once and keeps the outcome as bits, and the
// core-neighbour and tree-adjacency passes read bits.  adj[J * stride + k]
// (stride = ntile * kTile) holds row k's neighbours in column tile J: bit b of
// component i is the pair (k, J * kTile + 32 i + b).  Every decision is the
// FP32 predicate of the distance passes (the distance of (k, l) and of (l, k)
// is the same number), so the clusters are the same.

// v_writelane_b32: the returned register equals `old` except in lane `lane`,
// which takes the wave-uniform `v`
extern "C" __device__ int lane_write(int v, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

// 1b. pairs of the upper triangle of tiles (J >= I), each once.  Block (g, I)
// takes row tile I against the column tiles J >= I of group g (COLG tiles);
// with CS > 1, CS threads share a row, each taking 1/CS of every column tile.
// A thread's hits are its row's word of tile J; for J > I the wave's ballot of
// column t (that column's neighbours among the wave's 64 rows) is moved into
// lane t with writelane and stored as half of the column's word of tile I.
// Counts are the popcounts of both (exact, not capped at minPts).
template <int P, int COLG, int CS>
__global__ __launch_bounds__(kTile * CS) void k_adj(Cfg c, Bufs b, const float* __restrict__ zin, int Vin) {
  using ZT = typename ZVec<P>::T;
  constexpr int SPAN = kTile / CS, NW = SPAN / 32, NSET = (SPAN + 63) / 64;
  static_assert(SPAN % 32 == 0, "row words are 32-bit");
  __shared__ ZT s_z[kTile];
  __shared__ int s_cc[2][kTile];
  __shared__ int s_rc[CS][kTile];
  const int r = (int)(threadIdx.x & (kTile - 1)), q = (int)(threadIdx.x / kTile);
  const int lane = (int)(threadIdx.x & (kWave - 1)), half = r / kWave;
  const int V = dbscan_V(b, zin, Vin);
  const int nt = ntiles_of(V);
  const int I = (int)blockIdx.y, g = (int)blockIdx.x;
  const int J0 = max(g * COLG, I), J1 = min(g * COLG + COLG, nt);
  if (I >= nt || J0 >= J1) return;
  const ZT* z = reinterpret_cast<const ZT*>(zin ? zin : b.z);
  const size_t stride = (size_t)c.ntile * kTile;
  const int k = I * kTile + r;
  // rows past V sit at +1e30, columns past V at -1e30: no pair with either
  // is a hit (the squared distance overflows to infinity)
  const ZT zk = k < V ? z[k] : ZVec<P>::far();
  ZT zl[COLG];
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int l = (J0 + u) * kTile + r;
    zl[u] = (q == 0 && J0 + u < J1 && l < V) ? z[l] : ZVec<P>::nfar();
  }
  const float r2 = c.eps2;
  int cnt = 0;
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int J = J0 + u;
    if (J >= J1) break;
    if (u > 0) __syncthreads();  // the previous tile's readers are done
    if (q == 0) s_z[r] = zl[u];
    __syncthreads();
    uint32_t w[NW];
    int clo[NSET], chi[NSET];
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = 0u;
#pragma unroll
    for (int s = 0; s < NSET; ++s) clo[s] = chi[s] = 0;
#pragma unroll
    for (int t = 0; t < SPAN; ++t) {
      const bool h = ZVec<P>::d2(zk, s_z[q * SPAN + t]) <= r2;
      w[t >> 5] |= h ? (1u << (t & 31)) : 0u;
      const unsigned long long bal = __ballot(h);
      clo[t >> 6] = lane_write((int)(uint32_t)bal, t & 63, clo[t >> 6]);
      chi[t >> 6] = lane_write((int)(uint32_t)(bal >> 32), t & 63, chi[t >> 6]);
    }
    uint32_t* rw = reinterpret_cast<uint32_t*>(b.adj + (size_t)J * stride + k) + q * NW;
    if constexpr (NW == 4)
      *reinterpret_cast<uint4*>(rw) = make_uint4(w[0], w[1], w[2], w[3]);
    else if constexpr (NW == 2)
      *reinterpret_cast<uint2*>(rw) = make_uint2(w[0], w[1]);
    else
      rw[0] = w[0];
#pragma unroll
    for (int i = 0; i < NW; ++i) cnt += __popc(w[i]);
    if (J > I) {
#pragma unroll
      for (int s = 0; s < NSET; ++s) {
        const int t = 64 * s + lane;
        if (t < SPAN) {
          const int tc = q * SPAN + t;  // column within the tile
          uint2* cw = reinterpret_cast<uint2*>(b.adj + (size_t)I * stride + J * kTile + tc) + half;
          *cw = make_uint2((uint32_t)clo[s], (uint32_t)chi[s]);
          s_cc[half][tc] = __popc((uint32_t)clo[s]) + __popc((uint32_t)chi[s]);
        }
      }
      __syncthreads();
      if ((int)threadIdx.x < kTile) {
        const int l = J * kTile + (int)threadIdx.x;
        const int cc = s_cc[0][threadIdx.x] + s_cc[1][threadIdx.x];
        if (l < V && cc) atomicAdd(&b.ncount[l], cc);
      }
    }
  }
  if constexpr (CS > 1) {
    s_rc[q][r] = cnt;
    __syncthreads();
    if (q == 0)
#pragma unroll
      for (int i = 1; i < CS; ++i) cnt += s_rc[i][r];
  }
  if (q == 0 && k < V && cnt) atomicAdd(&b.ncount[k], cnt);
}

// 2b. lowest-index core neighbour from the bitmap.  A block takes 64 rows with
// kMcnSplit threads each.  The core flags of all V points go to LDS first
// (wave ballots of the counts); thread q of a row takes the column tiles q,
// q + kMcnSplit, ... (all its words requested at once) and keeps its lowest
// core hit, and the row's minimum is a butterfly over its kMcnSplit lanes.
// Also writes the rows' core and hook words (one 64-bit word per block).
__global__ __launch_bounds__(kMcnThreads) void k_mcn_bits(Cfg c, Bufs b, const float* __restrict__ zin,
                                                        int Vin) {
  constexpr int NWV = kMcnThreads / kWave;
  __shared__ unsigned long long s_core[kMaxWords];
  __shared__ int s_m[64];
  const int V = dbscan_V(b, zin, Vin);
  const int base = (int)blockIdx.x * 64;
  if (base >= V) return;
  const int lane = (int)(threadIdx.x & (kWave - 1)), wv = (int)(threadIdx.x / kWave);
  const int nt = ntiles_of(V);
  const size_t stride = (size_t)c.ntile * kTile;
  const int rr = (int)threadIdx.x / kMcnSplit, q = (int)threadIdx.x % kMcnSplit;
  const int k = base + rr;
  // the row words do not depend on the core flags: requested first
  uint4 a[kMcnLoads];
#pragma unroll
  for (int u = 0; u < kMcnLoads; ++u) {
    const int J = q + u * kMcnSplit;
    a[u] = (k < V && J < nt) ? b.adj[(size_t)J * stride + k] : make_uint4(0u, 0u, 0u, 0u);
  }
  const int nw = (V + 63) >> 6;
  for (int w0 = wv; w0 < nw; w0 += NWV * 8) {
    int n[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int pt = (w0 + u * NWV) * 64 + lane;
      n[u] = pt < V ? b.ncount[pt] : 0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const unsigned long long m = __ballot(n[u] >= c.min_pts);
      const int w = w0 + u * NWV;
      if (lane == 0 && w < nw) s_core[w] = m;
    }
  }
  __syncthreads();
  // descending, so the last hit kept is the one of the lowest tile (the
  // flag words past V may be stale in LDS: the row has no bit there)
  int m = kInt32Max;
#pragma unroll
  for (int u = kMcnLoads - 1; u >= 0; --u) {
    const int J = q + u * kMcnSplit;
    if (J >= nt) continue;
    const unsigned long long lo = (((unsigned long long)a[u].y << 32) | a[u].x) & s_core[2 * J];
    const unsigned long long hi = (((unsigned long long)a[u].w << 32) | a[u].z) & s_core[2 * J + 1];
    if (lo) m = J * kTile + __ffsll((long long)lo) - 1;
    else if (hi) m = J * kTile + 64 + __ffsll((long long)hi) - 1;
  }
#pragma unroll
  for (int off = 1; off < kMcnSplit; off <<= 1) m = min(m, __shfl_xor(m, off, kWave));
  if (q == 0) {
    if (k < V) b.mcn[k] = m;
    s_m[rr] = m;
  }
  __syncthreads();
  if (wv == 0) {
    const int kk = base + lane;
    const unsigned long long hk = __ballot(kk < V && s_m[lane] < kk);
    if (lane == 0) {
      b.hookmask[base >> 6] = hk;
      b.coremask[base >> 6] = s_core[base >> 6];
    }
  }
}

// 4b. tree adjacency from the bitmap: block (g, I) as in the distance pass
// (upper triangle of tiles, roots followed the same way).  For each column
// tile the block gathers, per tree, the mask of the tile's core columns in it
// (one ballot per tree present in a wave's 64 columns); a core row sets the
// bit of every other tree whose mask meets its word of the tile.
template <int COLG>
__global__ __launch_bounds__(kTile) void k_tree_adj_bits(Cfg c, Bufs b, const float* __restrict__ zin,
                                                         int Vin) {
  __shared__ int s_woff[kMaxWords];
  __shared__ unsigned long long s_rm[kMaxWords];
  __shared__ unsigned long long s_adj[kMaxTrees];
  __shared__ unsigned long long s_cm[kMaxTrees][2];
  __shared__ unsigned long long s_pres[2];
  const int V = dbscan_V(b, zin, Vin);
  const int nt = ntiles_of(V);
  const int I = (int)blockIdx.y, g = (int)blockIdx.x;
  const int J0 = max(g * COLG, I), J1 = min(g * COLG + COLG, nt);
  if (I >= nt || J0 >= J1) return;
  const size_t stride = (size_t)c.ntile * kTile;
  const int r = (int)threadIdx.x, lane = r & (kWave - 1), half = r / kWave;
  const int k = I * kTile + r;
  // every operand of the block is requested before the first wait
  uint4 aw[COLG];
  int ncl[COLG], rl[COLG];
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int J = J0 + u, l = J * kTile + r;
    const bool ok = J < J1 && l < V;
    aw[u] = (J < J1 && k < V) ? b.adj[(size_t)J * stride + k] : make_uint4(0u, 0u, 0u, 0u);
    ncl[u] = ok ? b.ncount[l] : 0;
    rl[u] = ok ? b.mcn[l] : -1;
  }
  const int nck = k < V ? b.ncount[k] : 0;
  const int hk = k < V ? b.mcn[k] : -1;
  constexpr int PERW = (kAdjMaxK / 64 + kTile - 1) / kTile;
  unsigned long long rw[PERW];
  int wlo, whi;
  root_words<kTile, PERW>(b, V, rw, wlo, whi);
  int rt[COLG + 1];
  rt[0] = nck >= c.min_pts ? hk : -1;
#pragma unroll
  for (int u = 0; u < COLG; ++u) rt[u + 1] = ncl[u] >= c.min_pts ? rl[u] : -1;
  follow_roots(b.mcn, rt);
  const int rk = rt[0];
  if (g * COLG <= I && I < g * COLG + COLG && k < V) b.root[k] = rk;
  const int R = tree_prefix_of<kTile, PERW>(rw, wlo, whi, s_woff, s_rm);
  if (R < 2 || R > kMaxTrees) return;
  if (threadIdx.x < kMaxTrees) s_adj[threadIdx.x] = 0ull;
  const int tk = nck >= c.min_pts ? tree_id(s_rm, s_woff, rk) : -1;
  unsigned long long mask = 0ull;
#pragma unroll
  for (int u = 0; u < COLG; ++u) {
    const int J = J0 + u;
    if (J >= J1) break;
    const int tl = ncl[u] >= c.min_pts ? tree_id(s_rm, s_woff, rt[u + 1]) : -1;
    __syncthreads();  // the previous tile's masks are read
    if (threadIdx.x < kMaxTrees) {
      s_cm[threadIdx.x][0] = 0ull;
      s_cm[threadIdx.x][1] = 0ull;
    }
    __syncthreads();
    {
      int rem = tl;
      unsigned long long pres = 0ull;
      while (true) {
        const unsigned long long act = __ballot(rem >= 0);
        if (!act) break;
        const int T = __shfl(rem, __ffsll((long long)act) - 1, kWave);
        const unsigned long long bal = __ballot(rem == T);
        if (lane == 0) s_cm[T][half] = bal;
        pres |= 1ull << T;
        if (rem == T) rem = -1;
      }
      if (lane == 0) s_pres[half] = pres;
    }
    __syncthreads();
    if (tk >= 0) {
      unsigned long long pres = (s_pres[0] | s_pres[1]) & ~(1ull << tk);
      const unsigned long long lo = ((unsigned long long)aw[u].y << 32) | aw[u].x;
      const unsigned long long hi = ((unsigned long long)aw[u].w << 32) | aw[u].z;
      while (pres) {
        const int T = __ffsll((long long)pres) - 1;
        pres &= pres - 1ull;
        if ((lo & s_cm[T][0]) | (hi & s_cm[T][1])) mask |= 1ull << T;
      }
    }
  }
  if (tk >= 0 && mask) atomicOr(&s_adj[tk], mask);
  __syncthreads();
  if (threadIdx.x < R && s_adj[threadIdx.x]) atomicOr(&b.tadj[threadIdx.x], s_adj[threadIdx.x]);
}

// 5. connected components of the tree graph and canonical cluster numbers
// (one 1024-thread block), or the exact fallback for more than 64 trees.
template <int P>
__device__ void uf_fallback(const Cfg& c, const Bufs& b, const float* zin, int V) {
  // single-workgroup union-find over core-core neighbour pairs.  root[]
  // already holds the hook forest of step 3 (each core points to a lower-index
  // core of its own component, roots point to themselves): a valid starting
  // forest.  Hooks always go to the smaller root, so the final root of a
  // component is its lowest core index.
  using ZT = typename ZVec<P>::T;
  const ZT* z = reinterpret_cast<const ZT*>(zin ? zin : b.z);
  int* parent = b.root;
  const float r2 = c.eps2;
  auto find = [&](int x) {
    while (true) {
      const int p = __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (p == x) return x;
      x = p;
    }
  };
  for (int a = threadIdx.x; a < V; a += kFinThreads) {
    if (b.ncount[a] < c.min_pts) continue;
    const ZT za = z[a];
    for (int l = a + 1; l < V; ++l) {
      if (b.ncount[l] < c.min_pts) continue;
      if (!(ZVec<P>::d2(za, z[l]) <= r2)) continue;
      int x = a, y = l;
      while (true) {
        x = find(x);
        y = find(y);
        if (x == y) break;
        if (x > y) {
          const int t = x;
          x = y;
          y = t;
        }
        int expected = y;
        if (__hip_atomic_compare_exchange_strong(&parent[y], &expected, x, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP))
          break;
        y = expected;
      }
    }
  }
  __syncthreads();
  for (int a = threadIdx.x; a < V; a += kFinThreads)
    if (b.ncount[a] >= c.min_pts) parent[a] = find(a);
  __syncthreads();
}

// Cluster statistics of Alg. 1 [Cluster stats] over one labelling chunk:
// count, cost sum, direction sums (for Eq. (16)) and minimum cost of every
// cluster.  Thread t holds the chunk's points a0 + u * kFinThreads + t (u
// ascending) and sums them in that order; the thread sums go through an xor
// butterfly within the wave, the wave results are added in wave order and
// the chunks in ascending order, so every run gives the same totals.  The
// running totals live in the cluster arrays: thread j < kStatClusters keeps
// clusters j, j + kStatClusters, ...
template <int P>
__device__ void chunk_stats(const Bufs& b, bool first, int M, const int (&lab)[kLabBatch],
                            const float (&Sa)[kLabBatch], const typename ZVec<P>::T (&ga)[kLabBatch],
                            float (*s_red)[kStatClusters][6], float (*s_tot)[6]) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  for (int c0 = 0; c0 < M; c0 += kStatClusters) {
    const int ncl = min(kStatClusters, M - c0);
    for (int j = 0; j < ncl; ++j) {
      const int cl = c0 + j;
      float sS = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, mn = INFINITY;
      int n = 0;
#pragma unroll
      for (int u = 0; u < kLabBatch; ++u) {
        const bool in = lab[u] == cl;
        n += __popcll(__ballot(in));
        if (in) {
          sS += Sa[u];
          g0 += ga[u].x;
          g1 += ga[u].y;
          if constexpr (P == 3) g2 += ga[u].z;
          mn = fminf(mn, Sa[u]);
        }
      }
      if (n) {  // wave-uniform
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
          sS += __shfl_xor(sS, off, kWave);
          g0 += __shfl_xor(g0, off, kWave);
          g1 += __shfl_xor(g1, off, kWave);
          if constexpr (P == 3) g2 += __shfl_xor(g2, off, kWave);
          mn = fminf(mn, __shfl_xor(mn, off, kWave));
        }
      }
      if (lane == 0) {
        float* r = s_red[w][j];
        r[0] = sS;
        r[1] = g0;
        r[2] = g1;
        r[3] = g2;
        r[4] = mn;
        r[5] = (float)n;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < ncl) {
      const int j = threadIdx.x, cl = c0 + j;
      float sS = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, mn = INFINITY;
      int n = 0;
      if (!first) {
        sS = b.c_cost[cl];
        g0 = b.c_dir[4 * cl];
        g1 = b.c_dir[4 * cl + 1];
        g2 = b.c_dir[4 * cl + 2];
        mn = b.c_smin[cl];
        n = b.c_size[cl];
      }
      for (int v = 0; v < kFinThreads / kWave; ++v) {
        const float* r = s_red[v][j];
        sS += r[0];
        g0 += r[1];
        g1 += r[2];
        g2 += r[3];
        mn = fminf(mn, r[4]);
        n += (int)r[5];
      }
      b.c_cost[cl] = sS;
      b.c_dir[4 * cl] = g0;
      b.c_dir[4 * cl + 1] = g1;
      b.c_dir[4 * cl + 2] = g2;
      b.c_smin[cl] = mn;
      b.c_size[cl] = n;
      if (c0 == 0) {  // the first kStatClusters clusters' totals stay in LDS for the means
        s_tot[j][0] = sS;
        s_tot[j][1] = g0;
        s_tot[j][2] = g1;
        s_tot[j][3] = g2;
        s_tot[j][5] = (float)n;
      }
    }
    __syncthreads();
  }
}

// Point data of one labelling chunk (points a0 + u * kFinThreads + threadIdx.x):
// neighbour count, the point whose root gives the label (itself if core,
// its lowest-index core neighbour if border, -1 if noise), and with stats
// its cost and direction.
template <int P>
__device__ __forceinline__ void label_loads(const Cfg& c, const Bufs& b, int a0, int V, bool stats,
                                            int (&nc)[kLabBatch], int (&x)[kLabBatch], float (&Sa)[kLabBatch],
                                            typename ZVec<P>::T (&ga)[kLabBatch]) {
  using ZT = typename ZVec<P>::T;
  const ZT* gv = reinterpret_cast<const ZT*>(b.gv);
#pragma unroll
  for (int u = 0; u < kLabBatch; ++u) {
    const int a = a0 + u * kFinThreads + threadIdx.x;
    nc[u] = a < V ? b.ncount[a] : 0;
    const int mc = a < V ? b.mcn[a] : kInt32Max;
    x[u] = a >= V ? -1 : (nc[u] >= c.min_pts ? a : (mc != kInt32Max ? mc : -1));
    Sa[u] = (stats && a < V) ? b.Sv[a] : 0.f;
    ga[u] = (stats && a < V) ? gv[a] : ZT{};
  }
}

template <int P>
__device__ __forceinline__ void tree_cc_body(const Cfg& c, const Bufs& b, int bx, int by, int nbx, const float* __restrict__ zin, int Vin, int* mout, int* lab_out, int* cnt_out) {
  using ZT = typename ZVec<P>::T;
  __shared__ int s_woff[kMaxWords];
  __shared__ unsigned long long s_rm[kMaxWords];
  __shared__ unsigned long long s_adj[kMaxTrees];
  __shared__ int s_tc[kMaxTrees];
  __shared__ int s_M;
  __shared__ float s_red[kFinThreads / kWave][kStatClusters][6];
  __shared__ float s_tot[kStatClusters][6];
  const int V = dbscan_V(b, zin, Vin);
  // the first labelling chunk's point data and roots do not depend on the
  // tree numbering or the closure: they are requested first, so their loads
  // overlap those steps (the union-find fallback rewrites the roots; it
  // reloads them)
  const bool stats_pts = zin == nullptr;
  int nc0[kLabBatch], x0[kLabBatch], r0[kLabBatch];
  float S0[kLabBatch];
  ZT g0[kLabBatch];
  label_loads<P>(c, b, 0, V, stats_pts, nc0, x0, S0, g0);
  unsigned long long rw[1];
  int wlo, whi;
  root_words<kFinThreads, 1>(b, V, rw, wlo, whi);
  const unsigned long long tadj0 = threadIdx.x < kMaxTrees ? b.tadj[threadIdx.x] : 0ull;
#pragma unroll
  for (int u = 0; u < kLabBatch; ++u) r0[u] = x0[u] >= 0 ? b.root[x0[u]] : -1;
  const int R = V > 0 ? tree_prefix_of<kFinThreads, 1>(rw, wlo, whi, s_woff, s_rm) : 0;
  const bool overflow = R > kMaxTrees;
  if (threadIdx.x == 0) {
    b.ctrl->n_trees = R;
    b.ctrl->tree_overflow = overflow ? 1 : 0;
    s_M = R <= 1 ? R : 0;
  }
  if (threadIdx.x < kMaxTrees) s_tc[threadIdx.x] = 0;
  __syncthreads();
  if (R >= 2 && !overflow) {
    // the tree graph: row t holds the trees adjacent to tree t (OR-ed by
    // the tree-adjacency blocks)
    if (threadIdx.x < R) s_adj[threadIdx.x] = tadj0;
    __syncthreads();
    if (threadIdx.x < kWave) {
      const int r = threadIdx.x;
      // make the relation symmetric, then close it transitively
      unsigned long long reach = r < R ? (s_adj[r] | (1ull << r)) : 0ull;
      for (int t = 0; t < R; ++t)
        if ((s_adj[t] >> r) & 1ull) reach |= 1ull << t;
      if (r >= R) reach = 0ull;
      for (int it = 0; it < 64; ++it) {
        unsigned long long nr = reach;
        for (int t = 0; t < R; ++t) {
          const unsigned long long rt = __shfl(reach, t, kWave);
          if ((reach >> t) & 1ull) nr |= rt;
        }
        const bool changed = __ballot(nr != reach) != 0ull;
        reach = nr;
        if (!changed) break;
      }
      const int cmin = r < R ? __ffsll((long long)reach) - 1 : kInt32Max;
      const unsigned long long heads = __ballot(r < R && cmin == r);
      if (r < R) {
        const unsigned long long below = cmin ? (heads & ((1ull << cmin) - 1ull)) : 0ull;
        s_tc[r] = __popcll(below);
      }
      if (r == 0) s_M = __popcll(heads);
    }
    __syncthreads();
  } else if (overflow) {
    // exact fallback; clusters = components ranked by their root (lowest core
    // index), the number of each root parked in label[root]
    uf_fallback<P>(c, b, zin, V);
#pragma unroll
    for (int u = 0; u < kLabBatch; ++u) r0[u] = x0[u] >= 0 ? b.root[x0[u]] : -1;
    int base = 0;
    for (int a0 = 0; a0 < V; a0 += kFinThreads) {
      const int a = a0 + threadIdx.x;
      const int isr = (a < V && b.ncount[a] >= c.min_pts && b.root[a] == a) ? 1 : 0;
      int tot;
      const int ex = block_excl_scan<kFinThreads>(isr, &tot);
      if (isr) b.label[a] = base + ex;
      base += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) s_M = base;
    __syncthreads();
  }
  const int M = s_M;
  if (threadIdx.x == 0) {
    b.ctrl->M = M;
    if (mout) *mout = M;
  }
  // labels: core -> cluster of its tree (or component), border -> cluster of
  // its lowest-index core neighbour, noise -> -1.  In the fallback the
  // cluster number of a root sits in label[root] and is never overwritten
  // (a root's own label is that same number).  Each thread takes kLabBatch
  // points at a time and issues all their loads before any store.  On the
  // feasible set of a replan the cluster statistics follow, chunk by chunk.
  const bool stats = stats_pts && M > 0;
  for (int a0 = 0; a0 < V; a0 += kFinThreads * kLabBatch) {
    int nc[kLabBatch], x[kLabBatch], r[kLabBatch], lab[kLabBatch];
    float Sa[kLabBatch];
    ZT ga[kLabBatch];
    if (a0 == 0) {
#pragma unroll
      for (int u = 0; u < kLabBatch; ++u) {
        nc[u] = nc0[u];
        x[u] = x0[u];
        r[u] = r0[u];
        Sa[u] = S0[u];
        ga[u] = g0[u];
      }
    } else {
      label_loads<P>(c, b, a0, V, stats_pts, nc, x, Sa, ga);
#pragma unroll
      for (int u = 0; u < kLabBatch; ++u) r[u] = x[u] >= 0 ? b.root[x[u]] : -1;
    }
#pragma unroll
    for (int u = 0; u < kLabBatch; ++u) {
      if (r[u] < 0) lab[u] = -1;
      else if (overflow) lab[u] = b.label[r[u]];
      else lab[u] = R == 1 ? 0 : s_tc[tree_id(s_rm, s_woff, r[u])];
    }
#pragma unroll
    for (int u = 0; u < kLabBatch; ++u) {
      const int a = a0 + u * kFinThreads + threadIdx.x;
      if (a >= V) continue;
      const bool core = nc[u] >= c.min_pts;
      if (!(overflow && core && r[u] == a)) b.label[a] = lab[u];
      if (lab_out) lab_out[a] = lab[u];
      if (cnt_out) cnt_out[a] = nc[u];
    }
    if (stats) chunk_stats<P>(b, a0 == 0, M, lab, Sa, ga, s_red, s_tot);
  }
  // means: cost (Alg. 1 [Cluster stats]) and normalised direction (Eq. (16)),
  // from the totals in LDS (clusters past kStatClusters from global memory)
  if (stats && (int)threadIdx.x < kStatClusters) {
    for (int cl = threadIdx.x; cl < M; cl += kStatClusters) {
      const bool lds = cl < kStatClusters;
      const float cnt = lds ? s_tot[cl][5] : (float)b.c_size[cl];
      const float sx = lds ? s_tot[cl][1] : b.c_dir[4 * cl], sy = lds ? s_tot[cl][2] : b.c_dir[4 * cl + 1];
      const float sz = lds ? s_tot[cl][3] : b.c_dir[4 * cl + 2];
      const float sc = lds ? s_tot[cl][0] : b.c_cost[cl];
      const float vx = sx / cnt, vy = sy / cnt;
      const float vz = P == 3 ? sz / cnt : 0.f;
      const float nv = sqrtf(__builtin_fmaf(vz, vz, __builtin_fmaf(vy, vy, vx * vx))) + c.norm_eps;
      b.c_cost[cl] = sc / cnt;
      b.c_dir[4 * cl] = vx / nv;
      b.c_dir[4 * cl + 1] = vy / nv;
      b.c_dir[4 * cl + 2] = P == 3 ? vz / nv : 0.f;
    }
  }
}

template <int P>
__global__ __launch_bounds__(kFinThreads) void k_tree_cc(Cfg c, Bufs b, const float* __restrict__ zin, int Vin, int* mout, int* lab_out, int* cnt_out) {
  tree_cc_body<P>(c, b, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, zin, Vin, mout, lab_out, cnt_out);
}

// ---------------------------------------------------------------------------
// DBSCAN on angular windows: single planners with 2-D features (exact,
// deterministic; the labels and statistics are those of the tiled passes).
//
// The features of Eq. (13) are unit directions scaled by |d| / (|d| + eps_n),
// so nearly all of them lie on the unit ring.  For two ring points with norms
// s, t in [s_lo, s_hi] and angular separation phi,
//   4 s_lo^2 sin^2(phi/2) <= |a - b|^2 = (s - t)^2 + 4 s t sin^2(phi/2)
//                         <= (s_hi - s_lo)^2 + 4 s_hi^2 sin^2(phi/2).
// With the error of the computed angles taken off, every ring point of a
// bucket inside the inner window of a point (u +- w_in in bucket units) is
// its neighbour and no ring point outside the outer window (u +- w_out) is.
// Only the ring points of the one or two buckets between the windows at each
// end, and the points off the ring, are decided by the distance test: the
// same FP32 expression as in every other DBSCAN pass, so the neighbour graph
// is the same, and so are the counts, the core flags and the labels.
//  bin    (in the compaction) each feature's bucket and its slot there
//  count  (K1, every block of k_wdbscan) the sorted order by bucket; count
//         = ring points of the inner window (two bucket starts) + hits among
//         the boundary buckets and the off-ring points: exact; the lowest
//         core index of every bucket
//  cc     (K2, the last block of k_wdbscan to finish K1) core buckets at most
//         w_g apart hold core points that are neighbours for certain, so a
//         run of such buckets is connected; two adjacent runs more than w_gout apart are not, and
//         runs in between are linked if one core pair across the gap is;
//         off-ring core points join through their own tests (union-find).
//         The lowest-index core neighbour of a non-core point is a range
//         minimum of the bucket minima over its inner window, then its
//         boundary buckets and the off-ring points.  Components are
//         numbered by their lowest core index; labels and cluster
//         statistics as in k_tree_cc.
// Work: O(V) window lookups and O(V * points of the boundary buckets) tests,
// against V^2 / 2 pair tests for the bitmap; one launch instead of four.

__device__ __forceinline__ int wmod(int j) { return j & (kWinBins - 1); }

// Buckets around a ring point at bucket coordinate u, as unwrapped indices
// (bucket j stands for j mod kWinBins): the inner window [sl, sh] and the
// boundary buckets [lb0, lb1], [rb0, rb1]; the three cover every bucket at
// most once.  all: the inner window is the whole circle.
struct WinRange {
  int sl, sh, lb0, lb1, rb0, rb1;
  bool all;
};
__device__ __forceinline__ WinRange win_range(const Cfg& c, float u) {
  WinRange r;
  r.sl = (int)ceilf(u - c.w_in);
  r.sh = (int)floorf(u + c.w_in) - 1;
  r.all = r.sh - r.sl + 1 >= kWinBins;
  if (r.sh < r.sl) r.sh = r.sl - 1;
  const int cl = (int)floorf(u - c.w_out), ch = (int)floorf(u + c.w_out);
  r.lb0 = max(cl, r.sh + 1 - kWinBins);
  r.lb1 = r.sl - 1;
  r.rb0 = r.sh + 1;
  r.rb1 = min(ch, r.lb0 + kWinBins - 1);
  return r;
}

// sorted positions of the buckets j0..j1 (unwrapped, at most kWinBins of
// them): [p0, p1) and [q0, q1)
__device__ __forceinline__ void win_pos(const int* __restrict__ ws, int j0, int j1, int& p0, int& p1,
                                        int& q0, int& q1) {
  p0 = p1 = q0 = q1 = 0;
  if (j1 < j0) return;
  const int n = j1 - j0 + 1, m = wmod(j0);
  p0 = ws[m];
  if (m + n <= kWinBins) {
    p1 = ws[m + n];
  } else {
    p1 = ws[kWinBins];
    q1 = ws[m + n - kWinBins];
  }
}

// the bucket of sorted position r (ring positions): the last bucket whose
// start is at most r
__device__ __forceinline__ int win_bucket_of(const int* s_start, int r) {
  int lo = 0, hi = kWinBins - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_start[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// unwrapped bucket range [lo, hi] (at most kWinBins buckets) holds bucket j
__device__ __forceinline__ bool win_in(int j, int lo, int hi) { return hi >= lo && wmod(j - lo) <= hi - lo; }

constexpr int kWinZone = 4096;    // zone points a count block keeps in LDS

// K1: counts and the sorted order.  Block i takes the sorted positions
// [i POS, i POS + POS) (sorted by bucket, then slot; off-ring points last),
// two threads per position.
//  - every block scans the bucket counts into LDS (block 0 publishes them);
//  - the block's zone: the buckets any of its ring points may find beyond
//    its inner window (the union of their boundary buckets) and the
//    off-ring points;
//  - one pass over every key places the block's own points and its zone
//    points at their sorted positions in LDS, with their features;
//  - count = ring points of the inner window (bucket starts) + distance
//    tests against the boundary buckets and the off-ring points, from LDS.
// A zone beyond kWinZone points keeps its indices in the block's region of
// a global array instead, and its features are read from global memory.
// The block's off-ring points are tested against every point by the whole
// block.  Writes the counts, the sorted features, indices and counts, and
// the lowest core index of every bucket (as kWinMaxK - index, an atomic
// maximum over zero-initialised words).  Called for count blocks bx that
// hold points (bx < ceil(V / POS)).
__device__ __forceinline__ void wcount_body(const Cfg& c, const Bufs& b, const float* __restrict__ zin, int V,
                                            int bx) {
  constexpr int NT = kFinThreads, POS = kWinPos, PER = kWinBins / NT;
  static_assert(NT == 2 * POS, "two threads per sorted position");
  __shared__ int s_start[kWinBins + 1];
  __shared__ int s_own[POS];     // own point: compacted index | bucket << kWinShift
  __shared__ float2 s_oz[POS];   // own point: feature
  __shared__ int s_half[POS];    // second half of each own point's count
  __shared__ union {
    int k[kWinZone];
    float2 z[kWinZone];
  } s_zn;                        // zone: indices, then features
  __shared__ int s_b01[2];
  const int R0 = bx * POS;
  const float2* z = reinterpret_cast<const float2*>(zin ? zin : b.z);
  const int t = (int)threadIdx.x;
  const int R1 = min(R0 + POS, V);
  // the first keys are requested with the bucket counts
  constexpr int KB = 16;  // keys per thread and round
  int key0[KB];
#pragma unroll
  for (int u = 0; u < KB; ++u) {
    const int k = u * NT + t;
    key0[u] = k < V ? b.wkey[k] : -1;
  }
  // bucket starts
  int cnt[PER], sum = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    cnt[i] = b.wcnt[t * PER + i];
    sum += cnt[i];
  }
  int nring;
  int off = block_excl_scan<NT>(sum, &nring);
  const int rr1 = min(R1, nring);
  // the buckets of the block's first and last ring points: the non-empty
  // buckets whose positions hold them
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int lo = off, hi = off + cnt[i];
    s_start[t * PER + i] = lo;
    if (lo <= R0 && R0 < hi) s_b01[0] = t * PER + i;
    if (lo <= rr1 - 1 && rr1 - 1 < hi) s_b01[1] = t * PER + i;
    off = hi;
  }
  if (t == 0) s_start[kWinBins] = nring;
  __syncthreads();
  if (bx == 0) {
#pragma unroll
    for (int i = 0; i < PER; ++i) b.wstart[t * PER + i] = s_start[t * PER + i];
    if (t == 0) {
      b.wstart[kWinBins] = nring;
      b.wstart[kWinBins + 1] = V;
    }
  }
  // The zone, block-uniform: one or two unwrapped bucket ranges [lo_g,
  // hi_g] (every boundary bucket of the block's ring points; the left
  // boundaries lie in range 0, the right ones in the last), stored from LDS
  // index base_g in unwrapped bucket order, then the off-ring points.
  int zlo[2] = {0, 0}, zhi[2] = {-1, -1}, zs0[2] = {0, 0}, zbase[2] = {0, 0};
  int nr = 0;
  if (R0 < rr1) {
    const int B0 = s_b01[0], B1 = s_b01[1];
    const int wo = (int)ceilf(c.w_out), wi = (int)floorf(c.w_in);
    zlo[0] = B0 - wo - 1;
    zhi[0] = B1 - wi + 1;
    zlo[1] = B0 + wi - 1;
    zhi[1] = B1 + wo + 2;
    nr = 2;
    if (zhi[1] - zlo[0] + 1 >= kWinBins) {
      zlo[0] = 0;
      zhi[0] = kWinBins - 1;
      nr = 1;
    } else if (zlo[1] <= zhi[0] + 1) {
      zhi[0] = zhi[1];
      nr = 1;
    }
    if (nr == 1) {
      zlo[1] = zlo[0];
      zhi[1] = zhi[0];
    }
  }
  // points of bucket range [lo, hi] (unwrapped, at most kWinBins buckets)
  auto npts = [&](int lo, int hi) {
    if (hi < lo) return 0;
    const int m = wmod(lo), x = m + (hi - lo) + 1;
    return x <= kWinBins ? s_start[x] - s_start[m] : nring - s_start[m] + s_start[x - kWinBins];
  };
  int zsize = 0;
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    zs0[g] = s_start[wmod(zlo[g])];
    zbase[g] = zsize;
    if (g < nr) zsize += npts(zlo[g], zhi[g]);
  }
  if (nr == 1) zbase[1] = zbase[0];
  const int zoff = zsize;  // the off-ring points
  zsize += R0 < rr1 ? V - nring : 0;
  const bool lds = zsize <= kWinZone;
  int* gzone = b.wzone + (size_t)bx * c.K;
  // zone index of the first point of unwrapped bucket j of range g
  auto zidx = [&](int g, int j) {
    const int m = wmod(zlo[g]), x = m + (j - zlo[g]);
    return zbase[g] + (x < kWinBins ? s_start[x] - zs0[g] : nring - zs0[g] + s_start[x - kWinBins]);
  };
  // own and zone points at their places: indices first, then every feature
  // gathered in one round
  for (int k0 = 0; k0 < V; k0 += NT * KB) {
    int key[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = k0 + u * NT + t;
      key[u] = k0 == 0 ? key0[u] : (k < V ? b.wkey[k] : -1);
    }
    // (straight-line per key: one LDS read, the rest arithmetic; the zone
    // index of a bucket's points follows from its position: bucket j at
    // offset d of range g starts at base_g + start(j) - start(lo_g), plus
    // the ring points when the range passes the end of the circle)
    int st[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) st[u] = s_start[key[u] < 0 ? 0 : min(key[u] >> kWinShift, kWinBins)];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      const int k = k0 + u * NT + t, bk = key[u] >> kWinShift, slot = key[u] & (kWinMaxK - 1);
      const int pos = st[u] + slot;
      const bool valid = key[u] >= 0;
      if (valid && pos >= R0 && pos < R1) s_own[pos - R0] = k | (bk << kWinShift);
      int zi = -1;
      if (bk == kWinBins) zi = zoff + slot;
#pragma unroll
      for (int g = 1; g >= 0; --g) {
        const int m = wmod(zlo[g]);
        if (g < nr && bk < kWinBins && wmod(bk - zlo[g]) <= zhi[g] - zlo[g])
          zi = zbase[g] - zs0[g] + pos + (bk < m ? nring : 0);
      }
      if (valid && R0 < rr1 && zi >= 0) {
        if (lds) s_zn.k[zi] = k;
        else gzone[zi] = k;
      }
    }
  }
  __syncthreads();
  {
    constexpr int ZPER = kWinZone / NT;
    const int nz = lds ? zsize : 0;
    int kz[ZPER];
#pragma unroll
    for (int j = 0; j < ZPER; ++j) kz[j] = j * NT + t < nz ? s_zn.k[j * NT + t] : -1;
    const int ko = t < POS && R0 + t < R1 ? s_own[t] & (kWinMaxK - 1) : -1;
    float2 zz[ZPER];
#pragma unroll
    for (int j = 0; j < ZPER; ++j) zz[j] = kz[j] >= 0 ? z[kz[j]] : make_float2(0.f, 0.f);
    const float2 zo = ko >= 0 ? z[ko] : make_float2(0.f, 0.f);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ZPER; ++j)
      if (kz[j] >= 0) s_zn.z[j * NT + t] = zz[j];
    if (t < POS) s_oz[t] = zo;
  }
  __syncthreads();
  // thread t works on position R0 + (t mod POS), half t / POS of its count
  const int pp = t & (POS - 1), half = t / POS;
  const int pos = R0 + pp;
  const bool own = pos < R1;
  const int ok = own ? s_own[pp] : 0;
  const int k = ok & (kWinMaxK - 1), bk = ok >> kWinShift;
  const float2 zk = own ? s_oz[pp] : make_float2(0.f, 0.f);
  const float r2 = c.eps2;
  const bool ring = pos < nring;
  // hits of zk among the zone entries [e0, e1)
  auto hits = [&](int e0, int e1) {
    int n = 0;
    if (lds) {
      int e = e0;
      for (; e + 4 <= e1; e += 4) {
        const float2 a0 = s_zn.z[e], a1 = s_zn.z[e + 1], a2 = s_zn.z[e + 2], a3 = s_zn.z[e + 3];
        n += (ZVec<2>::d2(zk, a0) <= r2 ? 1 : 0) + (ZVec<2>::d2(zk, a1) <= r2 ? 1 : 0) +
             (ZVec<2>::d2(zk, a2) <= r2 ? 1 : 0) + (ZVec<2>::d2(zk, a3) <= r2 ? 1 : 0);
      }
      for (; e < e1; ++e) n += ZVec<2>::d2(zk, s_zn.z[e]) <= r2 ? 1 : 0;
    } else {
      for (int e = e0; e < e1; e += 4) {
        int kq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) kq[u] = e + u < e1 ? gzone[e + u] : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (kq[u] >= 0) n += ZVec<2>::d2(zk, z[kq[u]]) <= r2 ? 1 : 0;
      }
    }
    return n;
  };
  // hits among the len buckets from bucket j0 (any representative) of zone
  // range g: one run of zone entries, or two where it passes the end of a
  // range that covers the whole circle
  auto range_hits = [&](int g, int j0, int len) {
    if (len <= 0) return 0;
    const int L = zhi[g] - zlo[g] + 1, d0 = wmod(j0 - zlo[g]);
    if (d0 + len <= L) return hits(zidx(g, zlo[g] + d0), zidx(g, zlo[g] + d0 + len));
    return hits(zidx(g, zlo[g] + d0), zidx(g, zlo[g] + L)) + hits(zidx(g, zlo[g]), zidx(g, zlo[g] + min(L, d0 + len - L)));
  };
  // half 0: the inner window and the left boundary (in zone range 0);
  // half 1: the right boundary (in the last range) and the off-ring points
  int n = 0;
  if (own && ring) {
    const WinRange r = win_range(c, win_u(c, zk));
    if (half == 0) {
      n = r.all ? nring : npts(r.sl, r.sh) + range_hits(0, r.lb0, r.lb1 - r.lb0 + 1);
    } else {
      if (!r.all) n = range_hits(1, r.rb0, r.rb1 - r.rb0 + 1);
      n += hits(zoff, zsize);
    }
  }
  if (half == 1) s_half[pp] = n;
  __syncthreads();
  if (half == 0) n += s_half[pp];
  // off-ring points of the block: every point, the whole block on each
  // (each thread tests a strided share of the features; a block sum)
  const int off0 = max(R0, nring), noff_own = max(0, R1 - off0);
  for (int i = 0; i < noff_own; ++i) {
    const float2 zo = s_oz[off0 - R0 + i];
    int h = 0;
    for (int q0 = t; q0 < V; q0 += NT * 4) {
      float2 zq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = q0 + u * NT;
        zq[u] = q < V ? z[q] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) h += (q0 + u * NT < V && ZVec<2>::d2(zo, zq[u]) <= r2) ? 1 : 0;
    }
    int tot;
    (void)block_excl_scan<NT>(h, &tot);
    if (half == 0 && pos == off0 + i) n = tot;
  }
  if (own && half == 0) {
    b.ncount[k] = n;
    b.wnc[pos] = n;
    reinterpret_cast<float2*>(b.zs)[pos] = zk;
    b.sid[pos] = k;
    if (ring && n >= c.min_pts) atomicMax(&b.wbmin[bk], kWinMaxK - k);
  }
}

// lowest index among the core neighbours of zk at sorted positions [p0, p1)
// (global sorted arrays)
__device__ __forceinline__ int win_core_min(float2 zk, const Bufs& b, int p0, int p1, float r2, int min_pts,
                                            int m) {
  const float2* zs = reinterpret_cast<const float2*>(b.zs);
  int q = p0;
  for (; q + 2 <= p1; q += 2) {
    const float2 a = zs[q], d = zs[q + 1];
    const int na = b.wnc[q], nd = b.wnc[q + 1];
    const int ia = b.sid[q], id = b.sid[q + 1];
    if (na >= min_pts && ZVec<2>::d2(zk, a) <= r2) m = min(m, ia);
    if (nd >= min_pts && ZVec<2>::d2(zk, d) <= r2) m = min(m, id);
  }
  if (q < p1 && b.wnc[q] >= min_pts && ZVec<2>::d2(zk, zs[q]) <= r2) m = min(m, b.sid[q]);
  return m;
}

constexpr int kNoCore = kWinMaxK;  // above every index (V <= kWinMaxK)

// Lowest-index core neighbour of one non-core point at feature zk, by the
// whole wave (zk and ring wave-uniform), as index | (bucket + 1) << kWinShift
// when its bucket is known (0 in the high bits otherwise), or kInt32Max if
// there is none.  Every core point of the inner window is a neighbour, so
// the window's lowest bucket minimum is the answer unless a boundary bucket
// holds a lower core index or there are off-ring points (LDS only); then
// the core points of the boundary buckets and the off-ring points are
// tested (every point for an off-ring zk).
__device__ int win_mcn_wave(const Cfg& c, const Bufs& b, const int* s_bmin, const int* ws, float2 zk, bool ring,
                            int nring, int V) {
  const int lane = (int)(threadIdx.x & (kWave - 1));
  const float2* zs = reinterpret_cast<const float2*>(b.zs);
  const float r2 = c.eps2;
  int m = kNoCore, mb = -1, mbnd = kNoCore;
  WinRange r{};
  if (ring) {
    r = win_range(c, win_u(c, zk));
    auto take = [&](int j) {
      const int v = s_bmin[wmod(j)];
      if (v < m) {
        m = v;
        mb = wmod(j);
      }
    };
    if (r.all) {
      for (int j = lane; j < kWinBins; j += kWave) take(j);
    } else {
      for (int j = r.sl + lane; j <= r.sh; j += kWave) take(j);
      for (int j = r.lb0 + lane; j <= r.lb1; j += kWave) mbnd = min(mbnd, (int)s_bmin[wmod(j)]);
      for (int j = r.rb0 + lane; j <= r.rb1; j += kWave) mbnd = min(mbnd, (int)s_bmin[wmod(j)]);
    }
    // (minimum over the wave; the bucket follows its index, which is unique)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int om = __shfl_xor(m, off, kWave), ob = __shfl_xor(mb, off, kWave);
      if (om < m) {
        m = om;
        mb = ob;
      }
      mbnd = min(mbnd, __shfl_xor(mbnd, off, kWave));
    }
    if (mbnd >= m && nring == V) return m >= kNoCore ? kInt32Max : (m | ((mb + 1) << kWinShift));
  }
  // the position ranges to test (all bounds requested together): the two
  // boundary sides (each up to two ranges) and the off-ring points, or every
  // point
  int p0[5] = {0, 0, 0, 0, 0}, p1[5] = {0, 0, 0, 0, 0};
  if (ring) {
    if (!r.all) {
      win_pos(ws, r.lb0, r.lb1, p0[0], p1[0], p0[1], p1[1]);
      win_pos(ws, r.rb0, r.rb1, p0[2], p1[2], p0[3], p1[3]);
    }
    p0[4] = nring;
    p1[4] = V;
  } else {
    p1[4] = V;
  }
  int mt = ring ? m : kNoCore;
  // one strided pass over the ranges laid end to end, four loads per lane
  // in flight
  int len[5], tot = 0;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    len[i] = max(0, p1[i] - p0[i]);
    tot += len[i];
  }
  auto at = [&](int e) {
    int q = -1;
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      if (q < 0 && e < len[i]) q = p0[i] + e;
      e -= len[i];
    }
    return q;
  };
  for (int e0 = lane; e0 < tot; e0 += 4 * kWave) {
    int qq[4], nq[4];
    float2 zq[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = e0 + u * kWave;
      qq[u] = e < tot ? at(e) : -1;
      nq[u] = qq[u] >= 0 ? b.wnc[qq[u]] : 0;
      zq[u] = qq[u] >= 0 ? zs[qq[u]] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (nq[u] >= c.min_pts && ZVec<2>::d2(zk, zq[u]) <= r2) mt = min(mt, b.sid[qq[u]]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mt = min(mt, __shfl_xor(mt, off, kWave));
  if (mt >= kNoCore) return kInt32Max;
  return mt == m && ring ? (m | ((mb + 1) << kWinShift)) : mt;
}

// union-find over the nodes of K2 (runs, then off-ring points), in global
// memory, within one workgroup: parents always point to a lower node.  Words
// that atomics update are read with atomic loads.
__device__ __forceinline__ int ld_wg(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ int win_find(int* parent, int x) {
  while (true) {
    const int p = ld_wg(&parent[x]);
    if (p == x) return x;
    x = p;
  }
}
__device__ __forceinline__ void win_union(int* parent, int x, int y) {
  while (true) {
    x = win_find(parent, x);
    y = win_find(parent, y);
    if (x == y) return;
    if (x > y) {
      const int t = x;
      x = y;
      y = t;
    }
    int expected = y;
    if (__hip_atomic_compare_exchange_strong(&parent[y], &expected, x, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
  }
}

// Point data of one labelling chunk of the window path (points a0 + u *
// kFinThreads + threadIdx.x): neighbour count and key; with stats the cost
// and direction.
__device__ __forceinline__ void win_label_keys(const Bufs& b, int a0, int V, int (&nc)[kLabBatch],
                                               int (&key)[kLabBatch]) {
#pragma unroll
  for (int u = 0; u < kLabBatch; ++u) {
    const int a = a0 + u * kFinThreads + threadIdx.x;
    nc[u] = a < V ? b.ncount[a] : 0;
    key[u] = a < V ? b.wkey[a] : -1;
  }
}
__device__ __forceinline__ void win_label_stats(const Bufs& b, int a0, int V, bool stats, float (&Sa)[kLabBatch],
                                                float2 (&ga)[kLabBatch]) {
  const float2* gv = reinterpret_cast<const float2*>(b.gv);
#pragma unroll
  for (int u = 0; u < kLabBatch; ++u) {
    const int a = a0 + u * kFinThreads + threadIdx.x;
    Sa[u] = (stats && a < V) ? b.Sv[a] : 0.f;
    ga[u] = (stats && a < V) ? gv[a] : float2{};
  }
}

// K2: one 1024-thread block.  Runs of core buckets, the links across their
// gaps and the off-ring core points give the components; the lowest-index
// core neighbour of each non-core point (one wave per point) gives the
// border rule; labels and cluster statistics as in k_tree_cc.  Clears the
// bucket counts and minima for the next call.
__device__ __forceinline__ void wcc_body(const Cfg& c, const Bufs& b, const float* __restrict__ zin, int V,
                                         int* mout, int* lab_out, int* cnt_out) {
  using ZT = float2;
  constexpr int PER = kWinBins / kFinThreads;  // buckets per thread
  constexpr int NBW = kWinMaxK / 32;           // words of the component-minimum bitmap
  constexpr int BPT = (NBW + kFinThreads - 1) / kFinThreads;  // of them per thread
  constexpr int NW = kFinThreads / kWave;
  static_assert(kWinMaxRuns <= kFinThreads, "one run per thread");
  __shared__ int s_lab[kWinBins];              // bucket -> run, then cluster label (-1: no core point)
  __shared__ int s_bmin[kWinBins];             // lowest core index of each bucket (kNoCore: none)
  __shared__ int s_run[kWinMaxRuns];           // run -> lowest core index, then cluster label
  __shared__ short s_mj[kWinMaxRuns], s_mp[kWinMaxRuns];  // gaps that may link two runs
  __shared__ unsigned s_bits[NBW];
  __shared__ int s_boff[NBW];
  __shared__ int s_nmaybe;
  __shared__ int s_ncl[kFinThreads];          // non-core points of one labelling round, then their results
  __shared__ float s_red[NW][kStatClusters][6];
  __shared__ float s_tot[kStatClusters][6];
  const int t = (int)threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  if (V == 0) {
    if (t == 0) {
      b.ctrl->n_trees = 0;
      b.ctrl->tree_overflow = 0;
      b.ctrl->M = 0;
      if (mout) *mout = 0;
    }
    return;
  }
  const bool stats_pts = zin == nullptr;
  const float2* zsrc = reinterpret_cast<const float2*>(zin ? zin : b.z);
  const float2* zs = reinterpret_cast<const float2*>(b.zs);
  const int* ws = b.wstart;
  const float r2 = c.eps2;
  // every independent operand first: the bucket minima and the first
  // labelling chunk's point data
  const int nring = ws[kWinBins];
  int bm[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int v = b.wbmin[t * PER + i];
    bm[i] = v ? kWinMaxK - v : kInt32Max;
  }
  int nc[kLabBatch], key[kLabBatch];
  win_label_keys(b, 0, V, nc, key);
  const int noff = V - nring;
  s_run[t] = kInt32Max;
#pragma unroll
  for (int i = 0; i < BPT; ++i)
    if (t * BPT + i < NBW) s_bits[t * BPT + i] = 0u;
  if (t == 0) s_nmaybe = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) s_bmin[t * PER + i] = min(bm[i], kNoCore);
  // the core bucket before each core bucket (cyclic) and the gap to it
  int mine = -1;
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if (bm[i] != kInt32Max) mine = t * PER + i;
  int last;
  int pv = block_excl_max<kFinThreads>(mine, &last);
  int st[PER], prv[PER], nst_mine = 0;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = t * PER + i;
    st[i] = 0;
    prv[i] = 0;
    if (bm[i] != kInt32Max) {
      prv[i] = pv >= 0 ? pv : last - kWinBins;
      st[i] = j - prv[i] > c.w_g ? 1 : 0;
      pv = j;
    }
    nst_mine += st[i];
  }
  int nst;
  const int st_before = block_excl_scan<kFinThreads>(nst_mine, &nst);
  const int nR = last < 0 ? 0 : max(nst, 1);
  // run of a core bucket: the starts at or before it, less one; the buckets
  // before the first start close the circle with the last run
  int cum = st_before;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = t * PER + i;
    if (bm[i] != kInt32Max) {
      cum += st[i];
      const int run = nst == 0 ? 0 : (cum > 0 ? cum - 1 : nst - 1);
      s_lab[j] = run;
      atomicMin(&s_run[run], bm[i]);
      if (st[i] && nR >= 2 && j - prv[i] <= c.w_gout) {
        const int q = atomicAdd(&s_nmaybe, 1);
        s_mj[q] = (short)j;
        s_mp[q] = (short)prv[i];
      }
    } else {
      s_lab[j] = -1;
    }
  }
  __syncthreads();
  const int nmaybe = s_nmaybe;
  const bool uf = nmaybe > 0 || noff > 0;
  const int stride = kWinMaxRuns + c.K;
  int* parent = b.wuf;
  int* cmin = b.wuf + stride;
  int* olab = b.wuf + 2 * stride;
  const int nn = nR + noff;  // union-find nodes: runs, then off-ring points by sorted position
  if (uf) {
    for (int i = t; i < nn; i += kFinThreads) {
      parent[i] = i;
      cmin[i] = i < nR ? s_run[i]
                       : (b.wnc[nring + i - nR] >= c.min_pts ? b.sid[nring + i - nR] : kInt32Max);
    }
    __syncthreads();
    // a gap that may link two runs: core pairs across it, one wave per gap
    for (int gi = wv; gi < nmaybe; gi += NW) {
      const int j = s_mj[gi], pj = s_mp[gi];
      int a0, a1, a2, a3, c0, c1, c2, c3;
      win_pos(ws, j - c.w_gout, pj, a0, a1, a2, a3);
      win_pos(ws, j, pj + c.w_gout, c0, c1, c2, c3);
      const int na = (a1 - a0) + (a3 - a2), nb = (c1 - c0) + (c3 - c2);
      // 64 points of each side per round, one per lane; the A points are
      // broadcast from their lanes
      bool hit = false;
      for (int ia0 = 0; ia0 < na && !hit; ia0 += kWave) {
        const int ia = ia0 + lane;
        const int pa = ia < a1 - a0 ? a0 + ia : a2 + ia - (a1 - a0);
        const bool ca = ia < na && b.wnc[pa] >= c.min_pts;
        const float2 za = ia < na ? zs[pa] : make_float2(0.f, 0.f);
        const unsigned long long acore = __ballot(ca);
        for (int ib0 = 0; ib0 < nb && !hit && acore; ib0 += kWave) {
          const int ib = ib0 + lane;
          const int pb = ib < c1 - c0 ? c0 + ib : c2 + ib - (c1 - c0);
          const bool cb = ib < nb && b.wnc[pb] >= c.min_pts;
          const float2 zb = ib < nb ? zs[pb] : make_float2(0.f, 0.f);
          bool h = false;
          unsigned long long am = acore;
          while (am) {
            const int L = __ffsll((long long)am) - 1;
            am &= am - 1ull;
            const float2 zl = make_float2(__shfl(za.x, L, kWave), __shfl(za.y, L, kWave));
            h |= cb && ZVec<2>::d2(zl, zb) <= r2;
          }
          hit = __ballot(h) != 0ull;
        }
      }
      if (hit && lane == 0) win_union(parent, s_lab[wmod(pj)], s_lab[j]);
    }
    // off-ring core points: every core neighbour, the whole block on each
    // (a thread unions each node it meets once in a row)
    for (int o = 0; o < noff; ++o) {
      const int po = nring + o;
      if (b.wnc[po] < c.min_pts) continue;
      const float2 zo = zs[po];
      int prev_node = -1;
      for (int q0 = t; q0 < V; q0 += kFinThreads * 4) {
        int nq[4];
        float2 zq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + u * kFinThreads;
          nq[u] = q < V ? b.wnc[q] : 0;
          zq[u] = q < V ? zs[q] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int q = q0 + u * kFinThreads;
          if (q >= V || q == po || nq[u] < c.min_pts || !(ZVec<2>::d2(zo, zq[u]) <= r2)) continue;
          const int node = q < nring ? s_lab[b.wkey[b.sid[q]] >> kWinShift] : nR + (q - nring);
          if (node != prev_node) win_union(parent, nR + o, node);
          prev_node = node;
        }
      }
    }
    __syncthreads();
    // (nodes that are not roots keep their own minimum; roots only decrease)
    for (int i = t; i < nn; i += kFinThreads) {
      const int rt = win_find(parent, i), m = ld_wg(&cmin[i]);
      if (m != kInt32Max && rt != i) atomicMin(&cmin[rt], m);
    }
    __syncthreads();
    for (int i = t; i < nn; i += kFinThreads) {
      const int m = ld_wg(&cmin[i]);
      if (ld_wg(&parent[i]) == i && m != kInt32Max) atomicOr(&s_bits[m >> 5], 1u << (m & 31));
    }
  } else if (nR > kWave && t < nR) {
    atomicOr(&s_bits[s_run[t] >> 5], 1u << (s_run[t] & 31));
  }
  __syncthreads();
  // clusters are the components ranked by their lowest core index
  int M;
  if (!uf && nR <= kWave) {
    // the runs are the components (at most one wave of them): a run's rank
    // is the number of runs with a lower minimum (the minima are distinct)
    M = nR;
    int r = 0;
    if (t < nR) {
      const int mv = s_run[t];
      for (int j = 0; j < nR; ++j) r += s_run[j] < mv ? 1 : 0;
    }
    __syncthreads();
    if (t < nR) s_run[t] = r;
  } else {
    int npop = 0;
#pragma unroll
    for (int i = 0; i < BPT; ++i) npop += t * BPT + i < NBW ? __popc(s_bits[t * BPT + i]) : 0;
    int boff = block_excl_scan<kFinThreads>(npop, &M);
#pragma unroll
    for (int i = 0; i < BPT; ++i)
      if (t * BPT + i < NBW) {
        s_boff[t * BPT + i] = boff;
        boff += __popc(s_bits[t * BPT + i]);
      }
    __syncthreads();
    auto rank_of = [&](int x) {
      const int w = x >> 5, bit = x & 31;
      return s_boff[w] + __popc(s_bits[w] & (bit ? (0xffffffffu >> (32 - bit)) : 0u));
    };
    if (t < nR) s_run[t] = rank_of(uf ? ld_wg(&cmin[win_find(parent, t)]) : s_run[t]);
    if (uf)
      for (int o = t; o < noff; o += kFinThreads)
        olab[o] = b.wnc[nring + o] >= c.min_pts ? rank_of(ld_wg(&cmin[win_find(parent, nR + o)])) : -1;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int j = t * PER + i;
    if (s_lab[j] >= 0) s_lab[j] = s_run[s_lab[j]];
  }
  if (t == 0) {
    b.ctrl->n_trees = nR;
    b.ctrl->tree_overflow = 0;
    b.ctrl->M = M;
    if (mout) *mout = M;
  }
  __syncthreads();
  // labels: core -> its component, border -> the component of its
  // lowest-index core neighbour, noise -> -1; statistics as in k_tree_cc
  const bool stats = stats_pts && M > 0;
  for (int a0 = 0; a0 < V; a0 += kFinThreads * kLabBatch) {
    int lab[kLabBatch];
    if (a0 > 0) win_label_keys(b, a0, V, nc, key);
    // (requested here, used by the statistics after the border rule)
    float Sa[kLabBatch];
    ZT ga[kLabBatch];
    win_label_stats(b, a0, V, stats_pts && M > 0, Sa, ga);
    // non-core points: the key of their lowest-index core neighbour (none:
    // noise).  They are listed in LDS, kFinThreads at a time, and every wave
    // takes list entries in turn, one point per wave.
    int mync = 0;
#pragma unroll
    for (int u = 0; u < kLabBatch; ++u) mync += (a0 + u * kFinThreads + t < V && nc[u] < c.min_pts) ? 1 : 0;
    int nnc;
    const int ncb = block_excl_scan<kFinThreads>(mync, &nnc);
    for (int base = 0; base < nnc; base += kFinThreads) {
      int r = ncb;
#pragma unroll
      for (int u = 0; u < kLabBatch; ++u) {
        const int a = a0 + u * kFinThreads + t;
        if (a < V && nc[u] < c.min_pts) {
          if (r >= base && r < base + kFinThreads) s_ncl[r - base] = a;
          ++r;
        }
      }
      __syncthreads();
      const int n_this = min(kFinThreads, nnc - base);
      for (int i = wv; i < n_this; i += NW) {
        const int a = s_ncl[i];
        const int ka = b.wkey[a];
        const int m = win_mcn_wave(c, b, s_bmin, ws, zsrc[a], (ka >> kWinShift) < kWinBins, nring, V);
        if (lane == 0) {
          b.mcn[a] = m == kInt32Max ? m : (m & (kWinMaxK - 1));
          s_ncl[i] = m;
        }
      }
      __syncthreads();
      // each owner takes its points' results
      r = ncb;
#pragma unroll
      for (int u = 0; u < kLabBatch; ++u) {
        const int a = a0 + u * kFinThreads + t;
        if (a < V && nc[u] < c.min_pts) {
          if (r >= base && r < base + kFinThreads) {
            // (the neighbour's bucket when known, else its key)
            const int m = s_ncl[r - base], mbk = (m >> kWinShift) - 1;
            key[u] = m == kInt32Max ? -1 : (mbk >= 0 ? mbk << kWinShift : b.wkey[m]);
          }
          ++r;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < kLabBatch; ++u) {
      const int bk = key[u] >> kWinShift;
      lab[u] = key[u] < 0 ? -1 : (bk < kWinBins ? s_lab[bk] : olab[key[u] & (kWinMaxK - 1)]);
    }
#pragma unroll
    for (int u = 0; u < kLabBatch; ++u) {
      const int a = a0 + u * kFinThreads + t;
      if (a >= V) continue;
      b.label[a] = lab[u];
      if (lab_out) lab_out[a] = lab[u];
      if (cnt_out) cnt_out[a] = nc[u];
    }
    if (stats) chunk_stats<2>(b, a0 == 0, M, lab, Sa, ga, s_red, s_tot);
  }
  if (stats && t < kStatClusters) {
    for (int cl = t; cl < M; cl += kStatClusters) {
      const bool lds = cl < kStatClusters;
      const float cnt = lds ? s_tot[cl][5] : (float)b.c_size[cl];
      const float sx = lds ? s_tot[cl][1] : b.c_dir[4 * cl], sy = lds ? s_tot[cl][2] : b.c_dir[4 * cl + 1];
      const float sc = lds ? s_tot[cl][0] : b.c_cost[cl];
      const float vx = sx / cnt, vy = sy / cnt;
      const float nv = sqrtf(__builtin_fmaf(vy, vy, vx * vx)) + c.norm_eps;
      b.c_cost[cl] = sc / cnt;
      b.c_dir[4 * cl] = vx / nv;
      b.c_dir[4 * cl + 1] = vy / nv;
      b.c_dir[4 * cl + 2] = 0.f;
    }
  }
  // the bucket counts and minima start from zero at the next call
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    b.wcnt[t * PER + i] = 0;
    b.wbmin[t * PER + i] = 0;
  }
  if (t == 0) b.wcnt[kWinBins] = 0;
}

// The window path in one launch: every block counts and places its share of
// the sorted positions (K1); the last block to finish, known from a
// completion ticket taken after a device-scope fence, then runs K2 on what
// every block wrote.  With no points only block 0 runs (K2's empty case).
__global__ __launch_bounds__(kFinThreads) void k_wdbscan(Cfg c, Bufs b, const float* __restrict__ zin, int Vin,
                                                         int* mout, int* lab_out, int* cnt_out) {
  __shared__ int s_last;
  const int V = dbscan_V(b, zin, Vin);
  if (V == 0) {
    if (blockIdx.x == 0) wcc_body(c, b, zin, 0, mout, lab_out, cnt_out);
    return;
  }
  const int nblk = (V + kWinPos - 1) / kWinPos;
  if ((int)blockIdx.x >= nblk) return;
  wcount_body(c, b, zin, V, (int)blockIdx.x);
  // every wave waits for its stores and atomics to reach the L2 of its XCD;
  // then one wave writes that L2 back (device-scope release) and takes a
  // ticket.  The block that takes the last one invalidates its caches
  // (device-scope acquire) and reads what every block wrote.
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    s_last = __hip_atomic_fetch_add(&b.ctrl->wticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nblk - 1;
    if (s_last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      b.ctrl->wticket = 0;  // for the next call
    }
  }
  __syncthreads();
  if (!s_last) return;
  wcc_body(c, b, zin, V, mout, lab_out, cnt_out);
}

// bucket and slot of caller features (stage calls; replans bin in the compaction)
__global__ __launch_bounds__(256) void k_wbin(Cfg c, Bufs b, const float* __restrict__ zin, int V) {
  const int a = (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (a >= V) return;
  win_bin(c, b, reinterpret_cast<const float2*>(zin)[a], a);
}

// ---------------------------------------------------------------------------
// Selection (Eq. (14), or Eq. (17)-(18) for the dynamic rule), computed the
// same way by every update block: each thread scans a strided subset of the
// clusters keeping its best and second-best key, then a fixed tree merges
// them (ties go to the lowest cluster number).
struct Sel {
  int sel, rule, h_used;
  uint32_t status_add;
  float margin, smin, v[3], vh[3];
};

// The statistics of cluster threadIdx.x come preloaded (pre_*: requested by
// the caller before the branch was known); further clusters are loaded here.
__device__ __forceinline__ Sel select_cluster(const Cfg& c, const Bufs& b, int M, float pre_cost, float pre_mn,
                                              float4 pre_dir) {
  __shared__ float s_k1[kUpdThreads / kWave], s_k2[kUpdThreads / kWave], s_m1[kUpdThreads / kWave];
  __shared__ int s_i1[kUpdThreads / kWave];
  const Ctrl* ct = b.ctrl;
  Sel s;
  s.sel = -1;
  s.rule = 0;
  s.h_used = 0;
  s.status_add = 0u;
  s.margin = INFINITY;
  s.smin = INFINITY;
  s.v[0] = s.v[1] = s.v[2] = s.vh[0] = s.vh[1] = s.vh[2] = 0.f;
  if (M == 0) {
    s.status_add = 4u;  // no cluster: update over all of V
    return s;
  }
  if (c.scene_mode == 1) {
    // the estimate of Eq. (17), computed once by the compaction kernel
    s.h_used = ct->dyn_h;
    s.v[0] = ct->v_obs[0];
    s.v[1] = ct->v_obs[1];
    s.v[2] = ct->v_obs[2];
    s.vh[0] = ct->v_hat[0];
    s.vh[1] = ct->v_hat[1];
    s.vh[2] = ct->v_hat[2];
    if (ct->dyn_ok) s.rule = 1;
    else s.status_add = 8u;
  }
  // best key (ties to the lowest cluster), its minimum cost, and the second
  // best key: per thread over a strided subset of the clusters, then wave
  // butterflies and the four waves in order (min and the tie rule are exact,
  // so the result does not depend on the combining order)
  float k1 = INFINITY, k2 = INFINITY, m1 = INFINITY;
  int i1 = kInt32Max;
  for (int cl = threadIdx.x; cl < M; cl += kUpdThreads) {
    const bool first = cl == (int)threadIdx.x;
    const float cost = first ? pre_cost : b.c_cost[cl], mn = first ? pre_mn : b.c_smin[cl];
    const float4 dir = first ? pre_dir : reinterpret_cast<const float4*>(b.c_dir)[cl];
    const float key = s.rule == 0 ? cost : dir.x * s.vh[0] + dir.y * s.vh[1] + dir.z * s.vh[2];
    if (key < k1) {  // clusters are visited in increasing order: strict < keeps the lowest
      k2 = k1;
      k1 = key;
      i1 = cl;
      m1 = mn;
    } else if (key < k2) {
      k2 = key;
    }
  }
  auto combine = [](float& a1, float& a2, int& ai, float& am, float b1, float b2, int bi, float bm) {
    const bool takeb = b1 < a1 || (b1 == a1 && bi < ai);
    const float n2 = fminf(fminf(a2, b2), takeb ? a1 : b1);
    a1 = takeb ? b1 : a1;
    ai = takeb ? bi : ai;
    am = takeb ? bm : am;
    a2 = n2;
  };
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const float b1 = __shfl_xor(k1, off, kWave), b2 = __shfl_xor(k2, off, kWave);
    const int bi = __shfl_xor(i1, off, kWave);
    const float bm = __shfl_xor(m1, off, kWave);
    combine(k1, k2, i1, m1, b1, b2, bi, bm);
  }
  const int wv = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_k1[wv] = k1;
    s_k2[wv] = k2;
    s_i1[wv] = i1;
    s_m1[wv] = m1;
  }
  __syncthreads();
  k1 = s_k1[0];
  k2 = s_k2[0];
  i1 = s_i1[0];
  m1 = s_m1[0];
#pragma unroll
  for (int w = 1; w < kUpdThreads / kWave; ++w) combine(k1, k2, i1, m1, s_k1[w], s_k2[w], s_i1[w], s_m1[w]);
  if (i1 >= M) {  // no key compared below +inf (infinite or NaN keys): the lowest cluster
    i1 = 0;
    m1 = b.c_smin[0];
  }
  s.sel = i1;
  s.smin = m1;
  s.margin = M > 1 ? k2 - k1 : INFINITY;
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// Weighted sums of one update block: wave w takes candidates w * PER ..
// w * PER + PER - 1 (in order), lane l the elements l, l + 64, ... (NCH
// chunks, two chunks of every row requested at once; a chunk past the row's
// end reads the next row, or the slack after the last, and is not used);
// element N m is the weight sum.  The four waves are added in order.
struct UpdLds {
  float w[kUpdChunk];
  int k[kUpdChunk];
  float acc[kUpdThreads / kWave][kFinChunks * kWave];
};

template <int NCH>
__device__ __forceinline__ void update_sums(const Bufs& b, int NM, float* part, UpdLds& L) {
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  constexpr int PER = kUpdChunk / (kUpdThreads / kWave);
#pragma unroll
  for (int c0 = 0; c0 < NCH; c0 += 2) {
    constexpr int CB = 2;
    float v[PER][CB];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const float* row = b.eps + (size_t)L.k[wv * PER + i] * NM + lane;
#pragma unroll
      for (int q = 0; q < CB; ++q) v[i][q] = c0 + q < NCH ? row[(c0 + q) * kWave] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < CB; ++q) {
      if (c0 + q >= NCH) break;
      const int e = (c0 + q) * kWave + lane;
      float acc = 0.f;
      if (e < NM) {
#pragma unroll
        for (int i = 0; i < PER; ++i) acc += L.w[wv * PER + i] * v[i][q];
      } else if (e == NM) {
#pragma unroll
        for (int i = 0; i < PER; ++i) acc += L.w[wv * PER + i];
      }
      L.acc[wv][e] = acc;
    }
  }
  __syncthreads();
  float (*s_acc)[kFinChunks * kWave] = L.acc;
  for (int e = threadIdx.x; e <= NM; e += kUpdThreads)
    part[e] = ((s_acc[0][e] + s_acc[1][e]) + s_acc[2][e]) + s_acc[3][e];
}

// Update partials, Eq. (19)-(20) (Eq. (6)-(7) on the fallback branches):
// block b takes kUpdChunk candidates (16 per wave); lane = element of the
// [N][m] sequence; the four waves' sums are combined in a fixed order.
template <int NCH>
__device__ __forceinline__ void update_body(const Cfg& c, const Bufs& b, UpdLds& L, int bx) {
  float* s_w = L.w;
  int* s_k = L.k;
  const Ctrl* ct = b.ctrl;
  // the candidate records of both branches are requested with the control
  // words, before the branch is known (every array holds K entries)
  const int a0 = bx * kUpdChunk;
  const int a = a0 + (int)threadIdx.x;
  const bool ina = threadIdx.x < kUpdChunk && a < c.K;
  const int ac = ina ? a : 0;  // unconditional loads at a clamped index
  const float S_all = b.S[ac];
  const int lab_v = b.label[ac], k_v = b.vidx[ac];
  const float S_v = b.Sv[ac];
  // and the statistics of cluster threadIdx.x, for the selection
  const int cq = (int)threadIdx.x < c.mcap ? (int)threadIdx.x : 0;
  const float pre_cost = b.c_cost[cq], pre_mn = b.c_smin[cq];
  const float4 pre_dir = reinterpret_cast<const float4*>(b.c_dir)[cq];
  const int branch = ct->branch;
  const bool bad = ct->nonfinite != 0;
  const int NM = c.NM;
  const bool over_all = branch != 0;
  const int M = branch == 0 ? ct->M : 0;
  const int ncand = over_all ? c.K : ct->n_feas;
  const bool mine = ina && !bad && a < ncand;
  int lab = -1, kk = 0;
  float Sa = 0.f;
  if (mine) {
    if (over_all) {
      kk = a;
      Sa = S_all;
    } else {
      lab = lab_v;
      kk = k_v;
      Sa = S_v;
    }
  }
  Sel s;
  if (branch == 0 && (a0 < ncand || bx == 0)) {
    s = select_cluster(c, b, M, pre_cost, pre_mn, pre_dir);
  } else {
    s.sel = -1;
    s.rule = 0;
    s.h_used = 0;
    s.status_add = 0u;
    s.margin = INFINITY;
    s.smin = INFINITY;
    for (int i = 0; i < 3; ++i) s.v[i] = s.vh[i] = 0.f;
  }
  if (bx == 0 && threadIdx.x == 0 && branch == 0) {
    Ctrl* cw = b.ctrl;
    cw->sel = s.sel;
    cw->rule = s.rule;
    cw->h_used = s.h_used;
    cw->margin = s.margin;
    cw->status = ct->status | s.status_add;
    for (int i = 0; i < 3; ++i) {
      cw->v_obs[i] = s.v[i];
      cw->v_hat[i] = s.vh[i];
    }
    cw->sel_size = s.sel >= 0 ? b.c_size[s.sel] : 0;
    cw->smin_sel = s.smin;
  }
  const int sel = s.sel;
  const float smin = over_all ? ct->smin_all : (sel >= 0 ? s.smin : ct->smin_feas);
  const float inv_l = 1.0f / c.lambda;
  if (threadIdx.x < kUpdChunk) {
    float w = 0.f;
    if (mine && (over_all || sel < 0 || lab == sel)) w = expf(-(Sa - smin) * inv_l);
    s_w[threadIdx.x] = w;
    s_k[threadIdx.x] = kk;  // a valid row whenever the weight is nonzero
  }
  __syncthreads();
  float* part = b.upart + (size_t)bx * (NM + 1);
  update_sums<NCH>(b, NM, part, L);
}

template <int NCH>
__global__ __launch_bounds__(kUpdThreads) void k_update(Cfg c, Bufs b) {
  __shared__ UpdLds L;
  update_body<NCH>(c, b, L, (int)blockIdx.x);
}

// Final combination (one block): sum of the update partials in a fixed order,
// U_new = U + sum / sum(w), outputs, shift (last control repeated), step
// counter and the info record.  NCH = ceil((N m + 1) / 64) element chunks.
struct FinLds {
  float part[kFinThreads / kWave][kMaxNM + 1];
  float tot[kMaxNM + 1];
  float un[kMaxNM];
};

template <int NCH>
__device__ __forceinline__ void finish_body(const Cfg& c, const Bufs& b, FinLds& sh, float* __restrict__ u_out, float* __restrict__ U_out, void* info_out) {
  float (*s_part)[kMaxNM + 1] = sh.part;
  float* s_tot = sh.tot;
  float* s_un = sh.un;
  // the control words and the nominal are requested with the partials
  const Ctrl cv = *b.ctrl;
  const bool bad = cv.nonfinite != 0;
  const int NM = c.NM, W = NM + 1;
  const int e_own = threadIdx.x;  // NM <= kMaxNM <= kFinThreads: one element per thread
  const int nb = c.nblk_upd;
  // wave w sums the rows w, w + 16, ... in increasing order, lane l the
  // elements l, l + 64, ... of each (whole rows: coalesced).  A batch of
  // kFinRows rows per wave is requested at once; rows past the last update
  // block are zero padding and the chunks past a row's end read the next
  // row (those sums are never used), so the loads need no tests.
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  constexpr int NW = kFinThreads / kWave;
  float acc[NCH];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) acc[ch] = 0.f;
  float u_own = 0.f;
  for (int r0 = wv; r0 < nb; r0 += NW * kFinRows) {
    float v[kFinRows][NCH];
#pragma unroll
    for (int rb = 0; rb < kFinRows; ++rb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) v[rb][ch] = b.upart[(r0 + rb * NW) * W + ch * kWave + lane];  // < 2^31
    if (r0 == wv) u_own = b.U[e_own < NM ? e_own : 0];
#pragma unroll
    for (int rb = 0; rb < kFinRows; ++rb)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) acc[ch] += v[rb][ch];
  }
  if (nb <= wv) u_own = b.U[e_own < NM ? e_own : 0];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int e = ch * kWave + lane;
    if (e < W) s_part[wv][e] = acc[ch];
  }
  __syncthreads();
  if (e_own < W) {
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w) t += s_part[w][e_own];
    s_tot[e_own] = t;
  }
  __syncthreads();
  const float wsum = s_tot[NM];
  if (e_own < NM) {
    const float un = bad ? u_own : u_own + s_tot[e_own] / wsum;
    if (U_out) U_out[e_own] = un;
    b.Unew[e_own] = un;
    s_un[e_own] = un;
  }
  __syncthreads();
  if (e_own < NM) {
    const int j = e_own / c.m, i = e_own % c.m;
    if (j == 0 && u_out) u_out[i] = s_un[e_own];
    if (!bad) {
      const int src = j + 1 < c.N ? j + 1 : c.N - 1;
      b.U[e_own] = s_un[src * c.m + i];
    }
  }
  if (threadIdx.x == 0) {
    Ctrl* cw = b.ctrl;
    const int branch = cv.branch;
    const bool cl = branch == 0;
    const bool hasM = cl && cv.M > 0;
    const float smin = !cl ? cv.smin_all : (hasM ? cv.smin_sel : cv.smin_feas);
    cw->wsum = wsum;
    // ring state for the next replan's rollout blocks
    cw->hs_head = cv.hist_head;
    cw->hs_count = cv.hist_count;
    cw->hs_nobs = cv.hist_nobs;
    if (!bad) {
      const uint32_t lo = cv.step_lo + 1u;
      cw->step_hi = lo == 0u ? cv.step_hi + 1u : cv.step_hi;
      cw->step_lo = lo;
    }
    if (info_out) {
      struct Info {
        int32_t branch, n_collide, n_feasible, n_ref, n_clusters, selected, selected_size, closest,
            rule, history_used;
        uint32_t status, step;
        float margin, s_min, ref_point[3], v_obs[3], v_obs_hat[3], weight_sum;
      };
      Info* inf = reinterpret_cast<Info*>(info_out);
      inf->branch = branch;
      inf->n_collide = bad ? 0 : cv.n_col;
      inf->n_feasible = bad ? 0 : cv.n_feas;
      inf->n_ref = cl ? cv.n_ref : 0;
      inf->n_clusters = cl ? cv.M : 0;
      inf->selected = hasM ? cv.sel : -1;
      inf->selected_size = hasM ? cv.sel_size : 0;
      inf->closest = cv.closest;
      inf->rule = hasM ? cv.rule : 0;
      inf->history_used = hasM ? cv.h_used : 0;
      inf->status = cv.status;
      inf->step = cv.step_used;
      inf->margin = hasM ? cv.margin : INFINITY;
      inf->s_min = smin;
      for (int i = 0; i < 3; ++i) {
        inf->ref_point[i] = cl ? cv.ref[i] : 0.f;
        inf->v_obs[i] = hasM ? cv.v_obs[i] : 0.f;
        inf->v_obs_hat[i] = hasM ? cv.v_hat[i] : 0.f;
      }
      inf->weight_sum = wsum;
    }
  }
}

template <int NCH>
__global__ __launch_bounds__(kFinThreads) void k_finish(Cfg c, Bufs b, float* __restrict__ u_out, float* __restrict__ U_out, void* info_out) {
  __shared__ FinLds sh;
  finish_body<NCH>(c, b, sh, u_out, U_out, info_out);
}

// ---------------------------------------------------------------------------
// Batched phases: persistent kernels over the work tables of a batch.  The
// DBSCAN tables depend on each planner's feasible count, so kb_plan fills
// them on the device after the compaction.

__global__ __launch_bounds__(kFinThreads) void kb_plan(CSlotStatic st, PlanOut o) {
  for (int kd = 0; kd < kPlanKinds; ++kd) {
    const int n = *o.n[kd];
    if (n == 0) continue;
    const int q = threadIdx.x;
    int ncnt = 0, nadj = 0;
    if (q < n) {
      const SlotStatic& S = *(const SlotStatic*)(st + o.slot[kd][q]);
      const Ctrl* ct = S.b.ctrl;
      const int V = ct->branch == 0 ? ct->n_feas : 0;
      if (kd == 2) {
        // angular windows: the count-and-place blocks
        ncnt = (V + kWinPos - 1) / kWinPos;
      } else {
        const int nt = ntiles_of(V);
        ncnt = nt * ((nt + o.colg - 1) / o.colg);
        nadj = nt * ((nt + kColGroup - 1) / kColGroup);
      }
    }
    int t1, t2;
    const int e1 = block_excl_scan<kFinThreads>(ncnt, &t1);
    const int e2 = block_excl_scan<kFinThreads>(nadj, &t2);
    if (q < n) {
      o.pref_cnt[kd][q] = e1;
      o.pref_adj[kd][q] = e2;
    }
    if (q == 0) {
      o.pref_cnt[kd][n] = t1;
      o.pref_adj[kd][n] = t2;
    }
  }
}

#define CEMPPI_SLOT(slot)                                     \
  const SlotStatic& S = *(const SlotStatic*)(st + (slot));    \
  const Cfg& c = S.c;                                         \
  const Bufs& b = S.b

template <int P, bool BIN = false>
__global__ __launch_bounds__(256) void kb_compact(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<256>(t, s_pref, [&](int slot, int local) {
    CEMPPI_SLOT(slot);
    compact_body<P, BIN>(c, b, local, 0, 0);
  });
}

// count / mcn items: local = I * ceil(nt / COLG) + g
template <int P>
__global__ __launch_bounds__(kFinThreads) void kb_sort(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kFinThreads>(t, s_pref, [&](int slot, int) {
    CEMPPI_SLOT(slot);
    sort_body<P>(c, b, nullptr, 0);
  });
}

template <int P, int COLG>
__global__ __launch_bounds__(kTile) void kb_count(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kTile>(t, s_pref, [&](int slot, int local) {
    CEMPPI_SLOT(slot);
    const int nt = ntiles_of(dbscan_V(b, nullptr, 0));
    const int ng = (nt + COLG - 1) / COLG;
    count_body<P, COLG, true>(c, b, local % ng, local / ng, 0, nullptr, 0);
  });
}

template <int P, int COLG>
__global__ __launch_bounds__(kTile) void kb_mcn(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kTile>(t, s_pref, [&](int slot, int local) {
    CEMPPI_SLOT(slot);
    const int nt = ntiles_of(dbscan_V(b, nullptr, 0));
    const int ng = (nt + COLG - 1) / COLG;
    mcn_body<P, COLG>(c, b, local % ng, local / ng, 0, nullptr, 0);
  });
}

template <int P>
__global__ __launch_bounds__(kTile) void kb_tree_adj(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kTile>(t, s_pref, [&](int slot, int local) {
    CEMPPI_SLOT(slot);
    const int nt = ntiles_of(dbscan_V(b, nullptr, 0));
    const int ng = (nt + kColGroup - 1) / kColGroup;
    tree_adj_body<P, true>(c, b, local % ng, local / ng, 0, nullptr, 0);
  });
}

// angular windows of the 2-D members: the count-and-place blocks of every
// member, then one block per member for the components and labels (the two
// phases of k_wdbscan as two launches)
__global__ __launch_bounds__(kFinThreads) void kb_wcount(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kFinThreads>(t, s_pref, [&](int slot, int local) {
    CEMPPI_SLOT(slot);
    wcount_body(c, b, nullptr, dbscan_V(b, nullptr, 0), local);
  });
}

__global__ __launch_bounds__(kFinThreads) void kb_wcc(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kFinThreads>(t, s_pref, [&](int slot, int) {
    CEMPPI_SLOT(slot);
    wcc_body(c, b, nullptr, dbscan_V(b, nullptr, 0), nullptr, nullptr, nullptr);
  });
}

template <int P>
__global__ __launch_bounds__(kFinThreads) void kb_tree_cc(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  for_each_item<kFinThreads>(t, s_pref, [&](int slot, int) {
    CEMPPI_SLOT(slot);
    tree_cc_body<P>(c, b, 0, 0, 0, nullptr, 0, nullptr, nullptr, nullptr);
  });
}

__global__ __launch_bounds__(kUpdThreads) void kb_update(CSlotStatic st, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  __shared__ UpdLds L;
  for_each_item<kUpdThreads>(t, s_pref, [&](int slot, int local) {
    CEMPPI_SLOT(slot);
    switch ((c.NM + 1 + kWave - 1) / kWave) {
      case 1: update_body<1>(c, b, L, local); break;
      case 2: update_body<2>(c, b, L, local); break;
      case 3: update_body<3>(c, b, L, local); break;
      case 4: update_body<4>(c, b, L, local); break;
      case 5: update_body<5>(c, b, L, local); break;
      default: update_body<6>(c, b, L, local); break;
    }
  });
}

__global__ __launch_bounds__(kFinThreads) void kb_finish(CSlotStatic st, CSlotIO io, Tab t) {
  __shared__ int s_pref[kMaxBatch + 1];
  __shared__ FinLds sh;
  for_each_item<kFinThreads>(t, s_pref, [&](int slot, int) {
    CEMPPI_SLOT(slot);
    const SlotIO& I = *(const SlotIO*)(io + slot);
    switch ((c.NM + 1 + kWave - 1) / kWave) {
      case 1: finish_body<1>(c, b, sh, I.u_out, I.U_out, I.info); break;
      case 2: finish_body<2>(c, b, sh, I.u_out, I.U_out, I.info); break;
      case 3: finish_body<3>(c, b, sh, I.u_out, I.U_out, I.info); break;
      case 4: finish_body<4>(c, b, sh, I.u_out, I.U_out, I.info); break;
      case 5: finish_body<5>(c, b, sh, I.u_out, I.U_out, I.info); break;
      default: finish_body<6>(c, b, sh, I.u_out, I.U_out, I.info); break;
    }
  });
}
#undef CEMPPI_SLOT

// ---------------------------------------------------------------------------
// launchers
// the angular-window path runs (single planners with 2-D features whose
// windows are valid; the no-allocation entry point has no window buffers)
static bool use_window(const Cfg& c, const Bufs& b) { return c.p == 2 && c.dbpath == 0 && b.wcnt; }

template <int P>
static void launch_dbscan_p(Launcher& L, const Cfg& c, const Bufs& b, const float* zin, int Vin,
                            int ntile, int* lab_out, int* cnt_out, int* mout) {
  if (P == 2 && use_window(c, b)) {
    // grid sized for every point the call may have (K for a replan)
    const int cap = ntile * kTile;
    L(k_wdbscan, dim3((cap + kWinPos - 1) / kWinPos), dim3(kFinThreads), c, b, zin, Vin, mout,
      lab_out, cnt_out);
    return;
  }
  const int ngrp = (ntile + kColGroup - 1) / kColGroup;
  const int ncnt = (ntile + kCntGroup - 1) / kCntGroup;
  dim3 tiles(ngrp, ntile), ctiles(ncnt, ntile);
  // planners of at most kSplitTiles tiles (K <= 4096) split every row over
  // kSplit threads: their few blocks would otherwise leave the loop latency
  // exposed; larger ones launch enough blocks, and more threads would cost
  // the branches that skip the passes
  if (b.adj && c.dbpath != 2) {
    // bitmap passes
    // one column tile per block and four threads per row at every size (A/B
    // on the clustering replan at K = 8192: 7.6 us against 8.3-16.4 us for
    // one or two threads per row or two or four tiles per block)
    const int nag = (ntile + kAdjGroup - 1) / kAdjGroup;
    L(k_adj<P, kAdjGroup, kSplit>, dim3(nag, ntile), dim3(kTile * kSplit), c, b, zin, Vin);
    L(k_mcn_bits, dim3(2 * ntile), dim3(kMcnThreads), c, b, zin, Vin);
    L(k_tree_adj_bits<kColGroup>, tiles, dim3(kTile), c, b, zin, Vin);
  } else if (c.ntile <= kSplitTiles) {
    const dim3 tb(kTile * kSplit);
    L(k_count<P, kSplit>, ctiles, tb, c, b, zin, Vin);
    L(k_mcn<P, kSplit>, ctiles, tb, c, b, zin, Vin);
    L(k_tree_adj<P, kSplit>, tiles, tb, c, b, zin, Vin);
  } else {
    const dim3 tb(kTile);
    L(k_count<P, 1>, ctiles, tb, c, b, zin, Vin);
    L(k_mcn<P, 1>, ctiles, tb, c, b, zin, Vin);
    L(k_tree_adj<P, 1>, tiles, tb, c, b, zin, Vin);
  }
  L(k_tree_cc<P>, dim3(1), dim3(kFinThreads), c, b, zin, Vin, mout, lab_out, cnt_out);
}

// Everything between the rollouts and the final combination, as one chain
// (a graph fork into a clustering and a fallback branch was measured slower:
// the cross-stream synchronisation of the branches costs more than the
// overlap saves).
void launch_post_rollout(Launcher& L, const Cfg& c, const Bufs& b) {
  const int nk = (c.K + 255) / 256;
  int* none = nullptr;
  if (c.p == 2) {
    if (use_window(c, b)) L(k_compact<2, true>, dim3(nk), dim3(256), c, b);
    else L(k_compact<2, false>, dim3(nk), dim3(256), c, b);
    launch_dbscan_p<2>(L, c, b, nullptr, 0, c.ntile, none, none, none);
  } else {
    L(k_compact<3, false>, dim3(nk), dim3(256), c, b);
    launch_dbscan_p<3>(L, c, b, nullptr, 0, c.ntile, none, none, none);
  }
  using UFn = void (*)(Cfg, Bufs);
  static const UFn upds[6] = {k_update<1>, k_update<2>, k_update<3>, k_update<4>, k_update<5>, k_update<6>};
  L(upds[(c.NM + 1 + kWave - 1) / kWave - 1], dim3(c.nblk_upd), dim3(kUpdThreads), c, b);
}

void launch_finish(Launcher& L, const Cfg& c, const Bufs& b, float* u_out, float* U_out, void* info) {
  static_assert(kFinChunks <= 6, "finish kernels exist for up to 6 element chunks");
  using FFn = void (*)(Cfg, Bufs, float*, float*, void*);
  static const FFn fins[6] = {k_finish<1>, k_finish<2>, k_finish<3>, k_finish<4>, k_finish<5>, k_finish<6>};
  L(fins[(c.NM + 1 + kWave - 1) / kWave - 1], dim3(1), dim3(kFinThreads), c, b, u_out, U_out, info);
}

void launch_stage_dbscan(Launcher& L, const Cfg& c, const Bufs& b, const float* z, int V,
                         int* ncount, int* label, int* mout) {
  // the stage runs on caller features: initialise the per-point arrays.  A
  // non-null feature pointer marks stage mode in the kernels.
  if (z == nullptr) z = b.z;
  if (V == 0) {
    // no points: only the cluster count (0) is produced
    if (c.p == 2)
      L(k_tree_cc<2>, dim3(1), dim3(kFinThreads), c, b, z, 0, mout, (int*)nullptr, (int*)nullptr);
    else
      L(k_tree_cc<3>, dim3(1), dim3(kFinThreads), c, b, z, 0, mout, (int*)nullptr, (int*)nullptr);
    return;
  }
  const int ntile = (V + kTile - 1) / kTile;
  L(k_init_points, dim3((V + 255) / 256), dim3(256), b, V);
  if (use_window(c, b)) L(k_wbin, dim3((V + 255) / 256), dim3(256), c, b, z, V);
  if (c.p == 2)
    launch_dbscan_p<2>(L, c, b, z, V, ntile, label, ncount, mout);
  else
    launch_dbscan_p<3>(L, c, b, z, V, ntile, label, ncount, mout);
}


template <int P>
static void launch_batch_dbscan(Launcher& L, const CSlotStatic cst, const BatchTabs& T, int kd) {
  const dim3 tb(kTile);
  switch (T.colg) {
    case 1:
      L(kb_count<P, 1>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      L(kb_mcn<P, 1>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      break;
    case 8:
      L(kb_count<P, 8>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      L(kb_mcn<P, 8>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      break;
    case 4:
      L(kb_count<P, 4>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      L(kb_mcn<P, 4>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      break;
    default:
      L(kb_count<P, 2>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      L(kb_mcn<P, 2>, dim3(T.grid_tile), tb, cst, T.cnt[kd]);
      break;
  }
}

void launch_batch_post(Launcher& L, const SlotStatic* st, const SlotIO* io, const BatchTabs& T) {
  const CSlotStatic cst = (CSlotStatic)st;
  const CSlotIO cio = (CSlotIO)io;
  for (int kd = 0; kd < kPlanKinds; ++kd) {
    if (!T.has[kd]) continue;
    if (kd == 0) L(kb_compact<2>, dim3(T.grid_compact[0]), dim3(256), cst, T.compact[0]);
    else if (kd == 1) L(kb_compact<3>, dim3(T.grid_compact[1]), dim3(256), cst, T.compact[1]);
    else L(kb_compact<2, true>, dim3(T.grid_compact[2]), dim3(256), cst, T.compact[2]);
  }
  L(kb_plan, dim3(1), dim3(kFinThreads), cst, T.plan);
  if (T.has[2]) {
    L(kb_wcount, dim3(T.grid_win), dim3(kFinThreads), cst, T.cnt[2]);
    L(kb_wcc, dim3(T.grid_cc[2]), dim3(kFinThreads), cst, T.cc[2]);
  }
  for (int kd = 0; kd < 2; ++kd) {
    if (!T.has[kd]) continue;
    if (kd == 0) L(kb_sort<2>, dim3(T.grid_cc[0]), dim3(kFinThreads), cst, T.cc[0]);
    else L(kb_sort<3>, dim3(T.grid_cc[1]), dim3(kFinThreads), cst, T.cc[1]);
  }
  for (int kd = 0; kd < 2; ++kd) {
    if (!T.has[kd]) continue;
    if (kd == 0) launch_batch_dbscan<2>(L, cst, T, 0);
    else launch_batch_dbscan<3>(L, cst, T, 1);
  }
  for (int kd = 0; kd < 2; ++kd) {
    if (!T.has[kd]) continue;
    if (kd == 0) L(kb_tree_adj<2>, dim3(T.grid_tile), dim3(kTile), cst, T.adj[0]);
    else L(kb_tree_adj<3>, dim3(T.grid_tile), dim3(kTile), cst, T.adj[1]);
  }
  for (int kd = 0; kd < 2; ++kd) {
    if (!T.has[kd]) continue;
    if (kd == 0) L(kb_tree_cc<2>, dim3(T.grid_cc[0]), dim3(kFinThreads), cst, T.cc[0]);
    else L(kb_tree_cc<3>, dim3(T.grid_cc[1]), dim3(kFinThreads), cst, T.cc[1]);
  }
  L(kb_update, dim3(T.grid_update), dim3(kUpdThreads), cst, T.update);
  L(kb_finish, dim3(T.grid_finish), dim3(kFinThreads), cst, cio, T.finish);
}

}  // namespace cemppi
