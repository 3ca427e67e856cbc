// batch.cpp -- batched form: one graph launch replans every member planner.
//
// The batch keeps, in one device allocation, a slot per member (its
// configuration and buffer pointers, copied at creation), the per-call
// input/output pointers, and the work tables of every phase.  Each phase is
// one persistent kernel per planner kind whose fixed grid walks the items of
// all members (see for_each_item), so the graph does not depend on what the
// members compute and is built once per tuning.
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
void launch_batch_rollout(Launcher& L, int kind, const SlotStatic* st, const SlotIO* io, Tab t,
                          int grid);
void launch_batch_post(Launcher& L, const SlotStatic* st, const SlotIO* io, const BatchTabs& T);
}  // namespace cemppi

using namespace cemppi;

struct ce_mppi_batch {
  int n = 0, device = 0, cus = 256;
  std::vector<ce_mppi_planner*> pl;
  void* dmem = nullptr;
  SlotStatic* d_st = nullptr;
  SlotIO* d_io = nullptr;
  SlotIO* h_io = nullptr;  // pinned staging of the per-call pointers
  std::vector<SlotIO> last_io;
  bool io_valid = false;
  bool upload_pending = false;
  hipEvent_t up_done = nullptr;
  Tab roll[3] = {};
  int roll_total[3] = {0, 0, 0};
  int compact_total[2] = {0, 0}, stats_total[2] = {0, 0}, update_total = 0;
  BatchTabs T{};
  ce_mppi_batch_tuning tune{2, 8, 4, 0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
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

void drop_graph(ce_mppi_batch* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  B->exec = nullptr;
  B->graph = nullptr;
}

int rollout_kind(const ce_mppi_planner* P) {
  if (P->c.dyn != 0) return 2;
  return P->c.seg == 32 ? 0 : 1;
}

void set_grids(ce_mppi_batch* B) {
  const int cus = B->cus;
  const ce_mppi_batch_tuning& t = B->tune;
  BatchTabs& T = B->T;
  for (int kd = 0; kd < 2; ++kd) {
    T.grid_compact[kd] = std::min(B->compact_total[kd], 4 * cus);
    T.grid_cc[kd] = std::min(T.cc[kd].n, cus);
    T.grid_stats[kd] = std::min(B->stats_total[kd], 4 * cus);
  }
  T.grid_tile = t.tile_blocks_per_cu * cus;
  T.grid_roots = 2 * cus;
  T.grid_update = std::min(B->update_total, 4 * cus);
  T.grid_finish = std::min(B->n, cus);
  T.colg = t.colg;
  T.plan.colg = t.colg;
}

hipError_t build_graph(ce_mppi_batch* B) {
  drop_graph(B);
  set_grids(B);
  hipError_t e = hipGraphCreate(&B->graph, 0);
  if (e != hipSuccess) return e;
  Launcher L(nullptr, B->graph);
  for (int k = 0; k < 3; ++k) {
    const int grid = std::min(B->roll_total[k], B->tune.roll_blocks_per_cu * B->cus);
    if (grid > 0) launch_batch_rollout(L, k, B->d_st, B->d_io, B->roll[k], grid);
  }
  launch_batch_post(L, B->d_st, B->d_io, B->T);
  if (L.err != hipSuccess) {
    drop_graph(B);
    return L.err;
  }
  e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) drop_graph(B);
  return e;
}

ce_status check_tuning(const ce_mppi_batch_tuning* t) {
  if (!t) return set_error(CE_EINVAL, "tuning is NULL");
  if (t->colg != 1 && t->colg != 2 && t->colg != 4)
    return set_error(CE_EINVAL, "colg must be 1, 2 or 4");
  if (t->tile_blocks_per_cu < 1 || t->tile_blocks_per_cu > 16)
    return set_error(CE_EINVAL, "tile_blocks_per_cu out of range 1..16");
  if (t->roll_blocks_per_cu < 1 || t->roll_blocks_per_cu > 8)
    return set_error(CE_EINVAL, "roll_blocks_per_cu out of range 1..8");
  if (t->reserved != 0) return set_error(CE_EINVAL, "reserved must be 0");
  return CE_OK;
}

ce_status to_slot_io(const ce_mppi_batch* B, const ce_mppi_batch_io* io, std::vector<SlotIO>& out) {
  out.resize(B->n);
  for (int i = 0; i < B->n; ++i) {
    const ce_mppi_batch_io& a = io[i];
    const ce_mppi_planner* P = B->pl[i];
    if (!a.x_t || !a.u_out) return set_error(CE_EINVAL, "batch io: x_t and u_out are required");
    if (a.reserved != 0) return set_error(CE_EINVAL, "batch io: reserved must be 0");
    if (a.n_obs < 0 || a.n_obs > P->c.max_obs)
      return set_error(CE_EINVAL, "batch io: n_obs out of range for member " + std::to_string(i));
    if (a.n_obs > 0 && !a.obstacles) return set_error(CE_EINVAL, "batch io: obstacles is NULL");
    SlotIO s{};
    s.x_t = a.x_t;
    s.obs = a.n_obs > 0 ? a.obstacles : nullptr;
    s.u_out = a.u_out;
    s.U_out = a.U_out;
    s.info = a.info;
    s.n_obs = a.n_obs;
    out[i] = s;
  }
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

  // slot lists and static tables (host), then one upload
  std::vector<int> ints;
  auto put = [&](const std::vector<int>& v) {
    const size_t off = ints.size();
    ints.insert(ints.end(), v.begin(), v.end());
    return off;
  };
  std::vector<int> lr[3], lp[2], all(n);
  for (int i = 0; i < n; ++i) {
    all[i] = i;
    lr[rollout_kind(planners[i])].push_back(i);
    lp[planners[i]->c.p == 2 ? 0 : 1].push_back(i);
  }
  auto prefix = [&](const std::vector<int>& list, auto items) {
    std::vector<int> p(list.size() + 1, 0);
    for (size_t q = 0; q < list.size(); ++q) p[q + 1] = p[q] + items(planners[list[q]]);
    return p;
  };
  size_t o_roll_slot[3], o_roll_pref[3];
  for (int k = 0; k < 3; ++k) {
    o_roll_slot[k] = put(lr[k]);
    const auto p = prefix(lr[k], [](const ce_mppi_planner* P) { return P->c.nblk_roll; });
    o_roll_pref[k] = put(p);
    B->roll_total[k] = p.back();
  }
  size_t o_p_slot[2], o_compact[2], o_cc[2], o_stats[2], o_cnt[2], o_adj[2], o_roots[2];
  for (int kd = 0; kd < 2; ++kd) {
    o_p_slot[kd] = put(lp[kd]);
    auto pc = prefix(lp[kd], [](const ce_mppi_planner* P) { return (P->c.K + 255) / 256; });
    o_compact[kd] = put(pc);
    B->compact_total[kd] = pc.back();
    o_cc[kd] = put(prefix(lp[kd], [](const ce_mppi_planner*) { return 1; }));
    auto ps = prefix(lp[kd], [](const ce_mppi_planner*) { return kStatItems; });
    o_stats[kd] = put(ps);
    B->stats_total[kd] = ps.back();
    const std::vector<int> zeros(lp[kd].size() + 1, 0);
    o_cnt[kd] = put(zeros);
    o_adj[kd] = put(zeros);
    o_roots[kd] = put(zeros);
  }
  const size_t o_all = put(all);
  auto pu = prefix(all, [](const ce_mppi_planner* P) { return P->c.nblk_upd; });
  const size_t o_update = put(pu);
  B->update_total = pu.back();
  const size_t o_finish = put(prefix(all, [](const ce_mppi_planner*) { return 1; }));

  const size_t st_bytes = ((sizeof(SlotStatic) * n + 255) / 256) * 256;
  const size_t io_bytes = ((sizeof(SlotIO) * n + 255) / 256) * 256;
  const size_t int_bytes = ints.size() * sizeof(int);
  hipError_t e = hipMalloc(&B->dmem, st_bytes + io_bytes + int_bytes);
  if (e != hipSuccess) {
    delete B;
    return set_error(CE_ENOMEM, std::string("batch table allocation failed: ") + hipGetErrorString(e));
  }
  char* base = static_cast<char*>(B->dmem);
  B->d_st = reinterpret_cast<SlotStatic*>(base);
  B->d_io = reinterpret_cast<SlotIO*>(base + st_bytes);
  int* di = reinterpret_cast<int*>(base + st_bytes + io_bytes);
  std::vector<SlotStatic> hs(n);
  for (int i = 0; i < n; ++i) {
    hs[i].c = planners[i]->c;
    hs[i].b = planners[i]->b;
  }
  e = hipMemcpy(B->d_st, hs.data(), sizeof(SlotStatic) * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(B->d_io, 0, io_bytes);
  if (e == hipSuccess) e = hipMemcpy(di, ints.data(), int_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&B->h_io), sizeof(SlotIO) * n, 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->up_done, hipEventDisableTiming);
  if (e != hipSuccess) {
    ce_mppi_batch_destroy(B);
    return set_hip_error(e, "batch_create");
  }
  for (int k = 0; k < 3; ++k)
    B->roll[k] = Tab{di + o_roll_slot[k], di + o_roll_pref[k], (int)lr[k].size()};
  BatchTabs& T = B->T;
  for (int kd = 0; kd < 2; ++kd) {
    const int nk = (int)lp[kd].size();
    const int* sl = di + o_p_slot[kd];
    T.compact[kd] = Tab{sl, di + o_compact[kd], nk};
    T.cc[kd] = Tab{sl, di + o_cc[kd], nk};
    T.stats[kd] = Tab{sl, di + o_stats[kd], nk};
    T.cnt[kd] = Tab{sl, di + o_cnt[kd], nk};
    T.adj[kd] = Tab{sl, di + o_adj[kd], nk};
    T.roots[kd] = Tab{sl, di + o_roots[kd], nk};
    T.plan.slot[kd] = sl;
    T.plan.n[kd] = nk;
    T.plan.pref_cnt[kd] = di + o_cnt[kd];
    T.plan.pref_adj[kd] = di + o_adj[kd];
    T.plan.pref_roots[kd] = di + o_roots[kd];
  }
  T.update = Tab{di + o_all, di + o_update, n};
  T.finish = Tab{di + o_all, di + o_finish, n};
  *out = B;
  return CE_OK;
}

void ce_mppi_batch_destroy(ce_mppi_batch* B) {
  if (!B) return;
  DeviceGuard guard(B->device);
  if (B->upload_pending) (void)hipEventSynchronize(B->up_done);
  drop_graph(B);
  if (B->up_done) (void)hipEventDestroy(B->up_done);
  if (B->h_io) (void)hipHostFree(B->h_io);
  if (B->dmem) (void)hipFree(B->dmem);
  delete B;
}

ce_status ce_mppi_batch_replan(ce_mppi_batch* B, const ce_mppi_batch_io* io, void* stream) {
  if (!B || !io) return set_error(CE_EINVAL, "NULL argument");
  std::vector<SlotIO> s;
  ce_status st = to_slot_io(B, io, s);
  if (st != CE_OK) return st;
  DeviceGuard guard(B->device);
  hipStream_t hs = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (!B->io_valid || std::memcmp(s.data(), B->last_io.data(), sizeof(SlotIO) * B->n) != 0) {
    // the staging buffer may still be read by the previous upload
    if (B->upload_pending) e = hipEventSynchronize(B->up_done);
    if (e == hipSuccess) {
      std::memcpy(B->h_io, s.data(), sizeof(SlotIO) * B->n);
      e = hipMemcpyAsync(B->d_io, B->h_io, sizeof(SlotIO) * B->n, hipMemcpyHostToDevice, hs);
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
  if (!B->exec) {
    e = build_graph(B);
    if (e != hipSuccess) return set_hip_error(e, "batch graph build");
  }
  e = hipGraphLaunch(B->exec, hs);
  if (e != hipSuccess) return set_hip_error(e, "batch graph launch");
  return CE_OK;
}

ce_status ce_mppi_batch_set_tuning(ce_mppi_batch* B, const ce_mppi_batch_tuning* t) {
  if (!B) return set_error(CE_EINVAL, "batch is NULL");
  ce_status st = check_tuning(t);
  if (st != CE_OK) return st;
  DeviceGuard guard(B->device);
  B->tune = *t;
  drop_graph(B);
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
  const int colgs[] = {1, 2, 4}, tiles[] = {2, 4, 8, 16}, rolls[] = {2, 4};
  for (int cg : colgs) {
    for (int tb : tiles) {
      for (int rb : rolls) {
        if (result != CE_OK) break;
        B->tune = ce_mppi_batch_tuning{cg, tb, rb, 0};
        drop_graph(B);
        // one untimed replan (builds the graph), then reps timed, each
        // candidate from the saved states
        result = restore();
        if (result == CE_OK) result = ce_mppi_batch_replan(B, io, stream);
        if (result == CE_OK) result = restore();
        if (result != CE_OK) break;
        e = hipEventRecord(e0, hs);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(B->exec, hs);
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
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  B->tune = result == CE_OK ? win : start;
  drop_graph(B);
  const ce_status rs = restore();
  if (result != CE_OK) return result;
  if (rs != CE_OK) return rs;
  if (best) *best = win;
  if (best_ms) *best_ms = win_ms;
  return CE_OK;
}

}  // extern "C"
