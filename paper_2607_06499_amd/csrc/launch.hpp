// launch.hpp -- one launch sequence, two ways to run it: kernels go either
// straight onto a stream or, while a graph is being built, into a chain of
// hipGraph kernel nodes (each depending on the previous one).  The recorded
// nodes keep their kernel, grid and block so that a node's arguments can be
// replaced later in the instantiated graph.
#pragma once

#include <hip/hip_runtime.h>

#include <tuple>
#include <utility>
#include <vector>

namespace cemppi {

struct Launcher {
  struct Node {
    hipGraphNode_t node;
    void* func;
    dim3 grid, block;
  };
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;  // non-null: record instead of launching
  std::vector<Node> nodes;
  hipError_t err = hipSuccess;

  explicit Launcher(hipStream_t s, hipGraph_t g = nullptr) : stream(s), graph(g) {}

  template <typename... Params, typename... Args>
  void operator()(void (*kernel)(Params...), dim3 grid, dim3 block, Args&&... args) {
    if (err != hipSuccess) return;
    if (!graph) {
      hipLaunchKernelGGL(kernel, grid, block, 0, stream, std::forward<Args>(args)...);
      err = hipGetLastError();
      return;
    }
    std::tuple<std::decay_t<Params>...> vals(std::forward<Args>(args)...);
    void* ptrs[sizeof...(Params) > 0 ? sizeof...(Params) : 1];
    fill(vals, ptrs, std::index_sequence_for<Params...>{});
    hipKernelNodeParams p{};
    p.func = reinterpret_cast<void*>(kernel);
    p.gridDim = grid;
    p.blockDim = block;
    p.sharedMemBytes = 0;
    p.kernelParams = ptrs;
    p.extra = nullptr;
    hipGraphNode_t node;
    hipGraphNode_t dep = nodes.empty() ? nullptr : nodes.back().node;
    err = hipGraphAddKernelNode(&node, graph, dep ? &dep : nullptr, dep ? 1 : 0, &p);
    if (err == hipSuccess) nodes.push_back(Node{node, p.func, grid, block});
  }

 private:
  template <typename Tup, size_t... I>
  static void fill(Tup& t, void** ptrs, std::index_sequence<I...>) {
    ((ptrs[I] = static_cast<void*>(&std::get<I>(t))), ...);
  }
};

// Replace the arguments of a recorded node in an instantiated graph.
template <typename... Vals>
hipError_t set_node_args(hipGraphExec_t exec, const Launcher::Node& n, Vals&... vals) {
  void* ptrs[] = {static_cast<void*>(&vals)...};
  hipKernelNodeParams p{};
  p.func = n.func;
  p.gridDim = n.grid;
  p.blockDim = n.block;
  p.sharedMemBytes = 0;
  p.kernelParams = ptrs;
  p.extra = nullptr;
  return hipGraphExecKernelNodeSetParams(exec, n.node, &p);
}

}  // namespace cemppi
