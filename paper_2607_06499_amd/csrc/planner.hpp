// planner.hpp -- host-side planner object shared by the single-planner and
// batched entry points (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "cemppi.h"
#include "device.hpp"
#include "launch.hpp"

namespace cemppi {

// Replan as a hipGraph: the whole kernel chain recorded once, the first
// (rollout) and last (finish) nodes re-pointed when the caller's buffers
// change.
struct ReplanGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Launcher::Node first{}, last{};
  const float* x = nullptr;
  const float* obs = nullptr;
  int n_obs = -1;
  float* u_out = nullptr;
  float* U_out = nullptr;
  void* info = nullptr;
};

// HIP-event timing of each replan: events before the rollout kernel, after
// it and after the final kernel.
struct Timing {
  int cap = 0, n = 0;
  std::vector<hipEvent_t> ev;
};

}  // namespace cemppi

struct ce_mppi_planner {
  ce_mppi_config cfg;
  cemppi::Cfg c;
  cemppi::Bufs b;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  size_t cap_K = 0;
  int launch_mode = CE_LAUNCH_GRAPH;
  cemppi::ReplanGraph g;
  cemppi::Timing t;
  // stream of the last replan (or batch replan) of this planner
  hipStream_t last_stream = nullptr;
  bool used = false;
};

namespace cemppi {

// Record the stream a planner was last replanned on (single or batched).
void mark_stream(ce_mppi_planner* P, hipStream_t s);

// ce_mppi_replan without the in-flight check, for callers that order the
// planner's replans themselves (the server); records the stream used.
ce_status replan_unchecked(ce_mppi_planner* P, const float* x_t, const float* obstacles, int32_t n_obs,
                           float* u_out, float* U_out, ce_mppi_info* info, hipStream_t s);

// Error reporting into the thread's last-error string (defined in capi.cpp).
ce_status set_error(ce_status s, const std::string& msg);
ce_status set_hip_error(hipError_t e, const char* what);

}  // namespace cemppi
