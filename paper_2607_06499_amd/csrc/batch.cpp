// batch.cpp -- batched form: one graph launch replans many member planners.
//
// The batch keeps one slot per member in device memory (its configuration
// and buffer pointers, copied at creation).  Every launch reads its work
// tables and per-member input/output pointers from an "area": area 0 holds
// the tables of the full member set (filled once); the other areas form a
// small ring for launches over member subsets (the tables are rebuilt on the
// host and uploaded with the pointers in one copy).  Each phase of the
// replan is one persistent kernel per planner kind whose fixed grid walks the
// items of all listed members (see for_each_item), so the graph of an area
// does not depend on which members a launch covers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "cemppi.h"
#include "device.hpp"
#include "launch.hpp"
#include "planner.hpp"

namespace cemppi {
void launch_batch_rollout(Launcher& L, int kind, int r, const SlotStatic* st, const SlotIO* io, Tab t,
                          int grid);
void launch_batch_post(Launcher& L, const SlotStatic* st, const SlotIO* io, const BatchTabs& T);
}  // namespace cemppi

using namespace cemppi;

namespace {

constexpr int kAreas = 4;  // area 0: the full member set; 1..3: subset ring

// Offsets (in ints) of every table inside an area, for n member capacity.
struct Layout {
  size_t cnt_roll[3], cnt_p[kPlanKinds], cnt_all;  // table counts n
  size_t roll_slot[3], roll_pref[3][4];
  size_t p_slot[kPlanKinds], compact[kPlanKinds], cc[kPlanKinds], dyn_cnt[kPlanKinds], dyn_adj[kPlanKinds];
  size_t all_slot, update, finish;
  size_t ints = 0;
  void make(int n) {
    size_t o = 0;
    auto take = [&](size_t k) {
      const size_t r = o;
      o += k;
      return r;
    };
    for (int k = 0; k < 3; ++k) cnt_roll[k] = take(1);
    for (int kd = 0; kd < kPlanKinds; ++kd) cnt_p[kd] = take(1);
    cnt_all = take(1);
    for (int k = 0; k < 3; ++k) {
      roll_slot[k] = take(n);
      for (int ri = 0; ri < 4; ++ri) roll_pref[k][ri] = take(n + 1);
    }
    for (int kd = 0; kd < kPlanKinds; ++kd) {
      p_slot[kd] = take(n);
      compact[kd] = take(n + 1);
      cc[kd] = take(n + 1);
      dyn_cnt[kd] = take(n + 1);
      dyn_adj[kd] = take(n + 1);
    }
    all_slot = take(n);
    update = take(n + 1);
    finish = take(n + 1);
    ints = o;
  }
};

struct Area {
  void* dmem = nullptr;  // SlotIO[n] then the tables
  SlotIO* d_io = nullptr;
  int* d_tab = nullptr;
  char* h_mem = nullptr;  // pinned mirror of the same layout
  size_t bytes = 0, io_bytes = 0;
  hipEvent_t done = nullptr;
  bool used = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchTabs T{};
  Tab roll[3][4] = {};
};

}  // namespace

struct ce_mppi_batch {
  int n = 0, device = 0, cus = 256;
  std::vector<ce_mppi_planner*> pl;
  std::vector<int> roll_kind, p_kind;
  bool has_roll[3] = {false, false, false};
  void* d_st_mem = nullptr;
  SlotStatic* d_st = nullptr;
  Layout lay;
  Area area[kAreas];
  int next_area = 1;
  // full-set uploads of area 0
  std::vector<SlotIO> last_io;
  bool io_valid = false;
  bool upload_pending = false;
  hipEvent_t up_done = nullptr;
  // totals of the full member set (upper bounds of any subset): grid sizes
  int roll_total[3][4] = {};
  int compact_total[kPlanKinds] = {}, update_total = 0, n_p[kPlanKinds] = {}, win_total = 0;
  ce_mppi_batch_tuning tune{8, 8, 4, 4};
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

int r_index(int r) { return r == 1 ? 0 : r == 2 ? 1 : r == 4 ? 2 : 3; }

int rollout_kind(const ce_mppi_planner* P) {
  if (P->c.dyn != 0) return 2;
  return P->c.seg == 32 ? 0 : 1;
}

void drop_graph(Area& a) {
  if (a.exec) (void)hipGraphExecDestroy(a.exec);
  if (a.graph) (void)hipGraphDestroy(a.graph);
  a.exec = nullptr;
  a.graph = nullptr;
}

void drop_graphs(ce_mppi_batch* B) {
  for (Area& a : B->area) drop_graph(a);
}

// Host tables of one member list (slot indices) in the area layout.
void fill_tables(const ce_mppi_batch* B, const int* members, int count, int* h) {
  const Layout& L = B->lay;
  std::vector<int> lr[3], lp[kPlanKinds];
  for (int q = 0; q < count; ++q) {
    const int s = members[q];
    lr[B->roll_kind[s]].push_back(s);
    lp[B->p_kind[s]].push_back(s);
  }
  auto prefix = [&](const std::vector<int>& list, size_t off, auto items) {
    h[off] = 0;
    for (size_t q = 0; q < list.size(); ++q) h[off + q + 1] = h[off + q] + items(B->pl[list[q]]);
  };
  auto copy = [&](const std::vector<int>& list, size_t off) {
    std::copy(list.begin(), list.end(), h + off);
  };
  for (int k = 0; k < 3; ++k) {
    h[L.cnt_roll[k]] = (int)lr[k].size();
    copy(lr[k], L.roll_slot[k]);
    for (int ri = 0; ri < 4; ++ri) {
      const int r = 1 << ri;
      prefix(lr[k], L.roll_pref[k][ri], [r](const ce_mppi_planner* P) {
        const int rpb = kRollWaves * (kWave / P->c.seg) * r;
        return (P->c.K + rpb - 1) / rpb;
      });
    }
  }
  for (int kd = 0; kd < kPlanKinds; ++kd) {
    h[L.cnt_p[kd]] = (int)lp[kd].size();
    copy(lp[kd], L.p_slot[kd]);
    prefix(lp[kd], L.compact[kd], [](const ce_mppi_planner* P) { return (P->c.K + 255) / 256; });
    prefix(lp[kd], L.cc[kd], [](const ce_mppi_planner*) { return 1; });
    // the DBSCAN tables are written on the device by kb_plan
  }
  h[L.cnt_all] = count;
  std::copy(members, members + count, h + L.all_slot);
  std::vector<int> all(members, members + count);
  prefix(all, L.update, [](const ce_mppi_planner* P) { return P->c.nblk_upd; });
  prefix(all, L.finish, [](const ce_mppi_planner*) { return 1; });
}

// Tables of an area as kernel arguments, with the grids of the tuning.
void area_tabs(const ce_mppi_batch* B, Area& a) {
  const Layout& L = B->lay;
  int* d = a.d_tab;
  for (int k = 0; k < 3; ++k)
    for (int ri = 0; ri < 4; ++ri)
      a.roll[k][ri] = Tab{d + L.roll_slot[k], d + L.roll_pref[k][ri], d + L.cnt_roll[k]};
  BatchTabs& T = a.T;
  const int cus = B->cus;
  for (int kd = 0; kd < kPlanKinds; ++kd) {
    const int* sl = d + L.p_slot[kd];
    const int* nk = d + L.cnt_p[kd];
    T.compact[kd] = Tab{sl, d + L.compact[kd], nk};
    T.cc[kd] = Tab{sl, d + L.cc[kd], nk};
    T.cnt[kd] = Tab{sl, d + L.dyn_cnt[kd], nk};
    T.adj[kd] = Tab{sl, d + L.dyn_adj[kd], nk};
    T.plan.slot[kd] = sl;
    T.plan.n[kd] = nk;
    T.plan.pref_cnt[kd] = d + L.dyn_cnt[kd];
    T.plan.pref_adj[kd] = d + L.dyn_adj[kd];
    T.has[kd] = B->n_p[kd] > 0;
    T.grid_compact[kd] = std::max(1, std::min(B->compact_total[kd], 4 * cus));
    T.grid_cc[kd] = std::max(1, std::min(B->n_p[kd], cus));
  }
  T.update = Tab{d + L.all_slot, d + L.update, d + L.cnt_all};
  T.finish = Tab{d + L.all_slot, d + L.finish, d + L.cnt_all};
  T.grid_tile = B->tune.tile_blocks_per_cu * cus;
  // count-and-place blocks of the angular windows: two per CU fit its LDS
  T.grid_win = std::max(1, std::min(B->win_total, 2 * cus));
  T.grid_update = std::max(1, std::min(B->update_total, 4 * cus));
  T.grid_finish = std::max(1, std::min(B->n, cus));
  T.colg = B->tune.colg;
  T.plan.colg = B->tune.colg;
}

hipError_t build_graph(ce_mppi_batch* B, Area& a) {
  drop_graph(a);
  area_tabs(B, a);
  hipError_t e = hipGraphCreate(&a.graph, 0);
  if (e != hipSuccess) return e;
  Launcher L(nullptr, a.graph);
  const int ri = r_index(B->tune.roll_per_wave);
  for (int k = 0; k < 3; ++k) {
    if (!B->has_roll[k]) continue;
    const int grid = std::max(1, std::min(B->roll_total[k][ri], B->tune.roll_blocks_per_cu * B->cus));
    launch_batch_rollout(L, k, B->tune.roll_per_wave, B->d_st, a.d_io, a.roll[k][ri], grid);
  }
  launch_batch_post(L, B->d_st, a.d_io, a.T);
  if (L.err != hipSuccess) {
    drop_graph(a);
    return L.err;
  }
  e = hipGraphInstantiate(&a.exec, a.graph, nullptr, nullptr, 0);
  if (e != hipSuccess) drop_graph(a);
  return e;
}

ce_status check_tuning(const ce_mppi_batch_tuning* t) {
  if (!t) return set_error(CE_EINVAL, "tuning is NULL");
  if (t->colg != 1 && t->colg != 2 && t->colg != 4 && t->colg != 8)
    return set_error(CE_EINVAL, "colg must be 1, 2, 4 or 8");
  if (t->tile_blocks_per_cu < 1 || t->tile_blocks_per_cu > 16)
    return set_error(CE_EINVAL, "tile_blocks_per_cu out of range 1..16");
  if (t->roll_blocks_per_cu < 1 || t->roll_blocks_per_cu > 8)
    return set_error(CE_EINVAL, "roll_blocks_per_cu out of range 1..8");
  if (t->roll_per_wave != 1 && t->roll_per_wave != 2 && t->roll_per_wave != 4 &&
      t->roll_per_wave != 8)
    return set_error(CE_EINVAL, "roll_per_wave must be 1, 2, 4 or 8");
  return CE_OK;
}

ce_status to_slot_io(const ce_mppi_planner* P, const ce_mppi_batch_io& a, int which, SlotIO& s) {
  if (!a.x_t || !a.u_out) return set_error(CE_EINVAL, "batch io: x_t and u_out are required");
  if (a.reserved != 0) return set_error(CE_EINVAL, "batch io: reserved must be 0");
  if (a.n_obs < 0 || a.n_obs > P->c.max_obs)
    return set_error(CE_EINVAL, "batch io: n_obs out of range for member " + std::to_string(which));
  if (a.n_obs > 0 && !a.obstacles) return set_error(CE_EINVAL, "batch io: obstacles is NULL");
  s = SlotIO{};
  s.x_t = a.x_t;
  s.obs = a.n_obs > 0 ? a.obstacles : nullptr;
  s.u_out = a.u_out;
  s.U_out = a.U_out;
  s.info = a.info;
  s.n_obs = a.n_obs;
  return CE_OK;
}

}  // namespace

extern "C" {

ce_status ce_mppi_batch_create(ce_mppi_planner* const* planners, int32_t n, ce_mppi_batch** out) {
  if (!out) return set_error(CE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!planners) return set_error(CE_EINVAL, "planners is NULL");
  if (n < 1 || n > CE_MPPI_MAX_BATCH) return set_error(CE_EINVAL, "batch size out of range 1..1024");
  std::set<const ce_mppi_planner*> seen;
  for (int i = 0; i < n; ++i) {
    if (!planners[i]) return set_error(CE_EINVAL, "NULL planner in batch");
    if (!seen.insert(planners[i]).second) return set_error(CE_EINVAL, "planner listed twice in batch");
    if (planners[i]->cfg.device != planners[0]->cfg.device)
      return set_error(CE_EINVAL, "batch members must share one device");
  }
  ce_mppi_batch* B = new (std::nothrow) ce_mppi_batch();
  if (!B) return set_error(CE_ENOMEM, "host allocation failed");
  B->n = n;
  B->device = planners[0]->cfg.device;
  B->pl.assign(planners, planners + n);
  DeviceGuard guard(B->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, B->device) == hipSuccess && prop.multiProcessorCount > 0)
    B->cus = prop.multiProcessorCount;
  B->roll_kind.resize(n);
  B->p_kind.resize(n);
  for (int i = 0; i < n; ++i) {
    const ce_mppi_planner* P = planners[i];
    B->roll_kind[i] = rollout_kind(P);
    // 2-D members on the angular windows (their path when the batch is
    // made) form a group of their own
    B->p_kind[i] = P->c.p == 3 ? 1 : (P->c.dbpath == 0 && P->b.wcnt ? 2 : 0);
    if (B->p_kind[i] == 2) B->win_total += (P->c.K + kWinPos - 1) / kWinPos;
    B->has_roll[B->roll_kind[i]] = true;
    B->n_p[B->p_kind[i]] += 1;
    for (int ri = 0; ri < 4; ++ri) {
      const int rpb = kRollWaves * (kWave / P->c.seg) * (1 << ri);
      B->roll_total[B->roll_kind[i]][ri] += (P->c.K + rpb - 1) / rpb;
    }
    B->compact_total[B->p_kind[i]] += (P->c.K + 255) / 256;
    B->update_total += P->c.nblk_upd;
  }
  B->lay.make(n);
  hipError_t e = hipMalloc(&B->d_st_mem, sizeof(SlotStatic) * n);
  if (e == hipSuccess) {
    B->d_st = static_cast<SlotStatic*>(B->d_st_mem);
    std::vector<SlotStatic> hs(n);
    for (int i = 0; i < n; ++i) {
      hs[i].c = planners[i]->c;
      hs[i].b = planners[i]->b;
    }
    e = hipMemcpy(B->d_st, hs.data(), sizeof(SlotStatic) * n, hipMemcpyHostToDevice);
  }
  for (int k = 0; k < kAreas && e == hipSuccess; ++k) {
    Area& a = B->area[k];
    a.io_bytes = ((sizeof(SlotIO) * n + 255) / 256) * 256;
    a.bytes = a.io_bytes + B->lay.ints * sizeof(int);
    e = hipMalloc(&a.dmem, a.bytes);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&a.h_mem), a.bytes, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&a.done, hipEventDisableTiming);
    if (e == hipSuccess) {
      a.d_io = static_cast<SlotIO*>(a.dmem);
      a.d_tab = reinterpret_cast<int*>(static_cast<char*>(a.dmem) + a.io_bytes);
      std::memset(a.h_mem, 0, a.bytes);
      e = hipMemset(a.dmem, 0, a.bytes);
    }
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->up_done, hipEventDisableTiming);
  if (e == hipSuccess) {
    // area 0: the full member set, once
    std::vector<int> all(n);
    for (int i = 0; i < n; ++i) all[i] = i;
    int* h = reinterpret_cast<int*>(B->area[0].h_mem + B->area[0].io_bytes);
    fill_tables(B, all.data(), n, h);
    e = hipMemcpy(B->area[0].d_tab, h, B->lay.ints * sizeof(int), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    ce_mppi_batch_destroy(B);
    return set_error(CE_ENOMEM, std::string("batch_create: ") + hipGetErrorString(e));
  }
  *out = B;
  return CE_OK;
}

void ce_mppi_batch_destroy(ce_mppi_batch* B) {
  if (!B) return;
  DeviceGuard guard(B->device);
  if (B->upload_pending) (void)hipEventSynchronize(B->up_done);
  for (Area& a : B->area) {
    if (a.used) (void)hipEventSynchronize(a.done);
    drop_graph(a);
    if (a.done) (void)hipEventDestroy(a.done);
    if (a.h_mem) (void)hipHostFree(a.h_mem);
    if (a.dmem) (void)hipFree(a.dmem);
  }
  if (B->up_done) (void)hipEventDestroy(B->up_done);
  if (B->d_st_mem) (void)hipFree(B->d_st_mem);
  delete B;
}

ce_status ce_mppi_batch_replan(ce_mppi_batch* B, const ce_mppi_batch_io* io, void* stream) {
  if (!B || !io) return set_error(CE_EINVAL, "NULL argument");
  std::vector<SlotIO> s(B->n);
  for (int i = 0; i < B->n; ++i) {
    ce_status st = to_slot_io(B->pl[i], io[i], i, s[i]);
    if (st != CE_OK) return st;
  }
  DeviceGuard guard(B->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  Area& a = B->area[0];
  hipError_t e = hipSuccess;
  if (!B->io_valid || std::memcmp(s.data(), B->last_io.data(), sizeof(SlotIO) * B->n) != 0) {
    // the staging buffer may still be read by the previous upload
    if (B->upload_pending) e = hipEventSynchronize(B->up_done);
    if (e == hipSuccess) {
      std::memcpy(a.h_mem, s.data(), sizeof(SlotIO) * B->n);
      e = hipMemcpyAsync(a.d_io, a.h_mem, sizeof(SlotIO) * B->n, hipMemcpyHostToDevice, hs);
    }
    if (e == hipSuccess) e = hipEventRecord(B->up_done, hs);
    if (e != hipSuccess) {
      B->io_valid = false;
      return set_hip_error(e, "batch io upload");
    }
    B->upload_pending = true;
    B->last_io = s;
    B->io_valid = true;
  }
  if (!a.exec) {
    e = build_graph(B, a);
    if (e != hipSuccess) return set_hip_error(e, "batch graph build");
  }
  e = hipGraphLaunch(a.exec, hs);
  if (e != hipSuccess) return set_hip_error(e, "batch graph launch");
  for (int i = 0; i < B->n; ++i) mark_stream(B->pl[i], hs);
  return CE_OK;
}

ce_status ce_mppi_batch_replan_subset(ce_mppi_batch* B, const int32_t* members, int32_t count,
                                      const ce_mppi_batch_io* io, void* stream) {
  if (!B || !members || !io) return set_error(CE_EINVAL, "NULL argument");
  if (count < 1 || count > B->n) return set_error(CE_EINVAL, "member count out of range");
  std::vector<char> seen(B->n, 0);
  std::vector<SlotIO> s(count);
  for (int q = 0; q < count; ++q) {
    const int m = members[q];
    if (m < 0 || m >= B->n) return set_error(CE_EINVAL, "member index out of range");
    if (seen[m]) return set_error(CE_EINVAL, "member listed twice");
    seen[m] = 1;
    ce_status st = to_slot_io(B->pl[m], io[q], m, s[q]);
    if (st != CE_OK) return st;
  }
  DeviceGuard guard(B->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  Area& a = B->area[B->next_area];
  B->next_area = B->next_area + 1 < kAreas ? B->next_area + 1 : 1;
  hipError_t e = hipSuccess;
  // the area's tables are in use until its previous launch has finished; the
  // wait polls the event (a blocking wait may give up the thread's time
  // slice, which shows up as millisecond latency spikes in a serving loop)
  if (a.used) {
    while ((e = hipEventQuery(a.done)) == hipErrorNotReady) {
    }
  }
  if (e != hipSuccess) return set_hip_error(e, "batch area wait");
  SlotIO* hio = reinterpret_cast<SlotIO*>(a.h_mem);
  for (int q = 0; q < count; ++q) hio[members[q]] = s[q];
  int* h = reinterpret_cast<int*>(a.h_mem + a.io_bytes);
  std::vector<int> mem(members, members + count);
  fill_tables(B, mem.data(), count, h);
  e = hipMemcpyAsync(a.dmem, a.h_mem, a.bytes, hipMemcpyHostToDevice, hs);
  if (e == hipSuccess && !a.exec) e = build_graph(B, a);
  if (e == hipSuccess) e = hipGraphLaunch(a.exec, hs);
  if (e == hipSuccess) e = hipEventRecord(a.done, hs);
  if (e != hipSuccess) return set_hip_error(e, "batch subset launch");
  a.used = true;
  for (int q = 0; q < count; ++q) mark_stream(B->pl[members[q]], hs);
  return CE_OK;
}

ce_status ce_mppi_batch_set_tuning(ce_mppi_batch* B, const ce_mppi_batch_tuning* t) {
  if (!B) return set_error(CE_EINVAL, "batch is NULL");
  ce_status st = check_tuning(t);
  if (st != CE_OK) return st;
  DeviceGuard guard(B->device);
  for (Area& a : B->area)
    if (a.used) (void)hipEventSynchronize(a.done);
  B->tune = *t;
  drop_graphs(B);
  return CE_OK;
}

ce_status ce_mppi_batch_get_tuning(const ce_mppi_batch* B, ce_mppi_batch_tuning* t) {
  if (!B || !t) return set_error(CE_EINVAL, "NULL argument");
  *t = B->tune;
  return CE_OK;
}

ce_status ce_mppi_batch_autotune(ce_mppi_batch* B, const ce_mppi_batch_io* io, int32_t reps,
                                 void* stream, ce_mppi_batch_tuning* best, double* best_ms) {
  if (!B || !io) return set_error(CE_EINVAL, "NULL argument");
  if (reps < 1 || reps > 1000) return set_error(CE_EINVAL, "reps out of range 1..1000");
  DeviceGuard guard(B->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  // save every member's state
  std::vector<std::vector<char>> saved(B->n);
  for (int i = 0; i < B->n; ++i) {
    size_t bytes = 0;
    ce_status st = ce_mppi_state_size(B->pl[i], &bytes);
    if (st == CE_OK) {
      saved[i].resize(bytes);
      st = ce_mppi_get_state(B->pl[i], saved[i].data(), bytes, stream);
    }
    if (st != CE_OK) return st;
  }
  auto restore = [&]() -> ce_status {
    for (int i = 0; i < B->n; ++i) {
      ce_status st = ce_mppi_set_state(B->pl[i], saved[i].data(), saved[i].size(), stream);
      if (st != CE_OK) return st;
    }
    return CE_OK;
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return set_hip_error(e, "autotune events");
  const ce_mppi_batch_tuning start = B->tune;
  ce_mppi_batch_tuning win = start;
  double win_ms = 1e300;
  ce_status result = CE_OK;
  // stage 1: rollout shape with the current DBSCAN shape; stage 2: DBSCAN
  // shape with the best rollout shape
  std::vector<ce_mppi_batch_tuning> cand;
  for (int r : {1, 2, 4, 8})
    for (int rb : {2, 4}) cand.push_back({start.colg, start.tile_blocks_per_cu, rb, r});
  for (int stage = 0; stage < 2 && result == CE_OK; ++stage) {
    if (stage == 1) {
      cand.clear();
      for (int cg : {2, 4, 8})
        for (int tb : {4, 8, 16}) cand.push_back({cg, tb, win.roll_blocks_per_cu, win.roll_per_wave});
    }
    for (const ce_mppi_batch_tuning& tc : cand) {
      B->tune = tc;
      drop_graphs(B);
      // one untimed replan (builds the graph), then reps timed, each
      // candidate from the saved states
      result = restore();
      if (result == CE_OK) result = ce_mppi_batch_replan(B, io, stream);
      if (result == CE_OK) result = restore();
      if (result != CE_OK) break;
      e = hipEventRecord(e0, hs);
      for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(B->area[0].exec, hs);
      if (e == hipSuccess) e = hipEventRecord(e1, hs);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        result = set_hip_error(e, "autotune timing");
        break;
      }
      const double per = (double)ms / reps;
      if (per < win_ms) {
        win_ms = per;
        win = B->tune;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  B->tune = result == CE_OK ? win : start;
  drop_graphs(B);
  const ce_status rs = restore();
  if (result != CE_OK) return result;
  if (rs != CE_OK) return rs;
  if (best) *best = win;
  if (best_ms) *best_ms = win_ms;
  return CE_OK;
}

}  // extern "C"
