// noalloc.hip -- DBSCAN on caller features without any allocation: the same
// kernels as ce_mppi_stage_dbscan, with their per-point work arrays carved out
// of one file-scope device array instead of a planner's arena.  For callers
// that cannot allocate device memory (graph capture, tight serving loops).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "cemppi.h"
#include "device.hpp"
#include "launch.hpp"
#include "planner.hpp"

namespace cemppi {
void launch_stage_dbscan(Launcher& L, const Cfg& c, const Bufs& b, const float* z, int V,
                         int* ncount, int* label, int* mout);

namespace {

constexpr size_t kMaxPts = CE_MPPI_NOALLOC_MAX_POINTS;
constexpr size_t al(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kWords = (kMaxPts + 63) / 64 + 1;
// byte offsets of the work arrays inside the scratch array
constexpr size_t o_ctrl = 0;
constexpr size_t o_ncount = o_ctrl + al(sizeof(Ctrl));
constexpr size_t o_mcn = o_ncount + al(4 * kMaxPts);
constexpr size_t o_root = o_mcn + al(4 * kMaxPts);
constexpr size_t o_label = o_root + al(4 * kMaxPts);
constexpr size_t o_core = o_label + al(4 * kMaxPts);
constexpr size_t o_hook = o_core + al(8 * kWords);
constexpr size_t o_tadj = o_hook + al(8 * kWords);
constexpr size_t o_pack = o_tadj + al(8 * kMaxTrees);  // [kMaxPts] float4 rows of 3-D features
constexpr size_t kScratchBytes = o_pack + al(16 * kMaxPts);

// The scratch array.  Host code never uses this name as an address: the
// device address of each GPU's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of this GPU's scratch array (looked up once per device, with
// that device current)
ce_status scratch_of(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return set_error(CE_EUNSUPPORTED, "device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return set_hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(CE_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_ptr[dev]);
  return CE_OK;
}

// [V][3] rows -> float4 rows (the kernels' 3-D layout)
__global__ __launch_bounds__(256) void k_pack3(const float* __restrict__ z, int V, float4* __restrict__ out) {
  const int a = blockIdx.x * 256 + threadIdx.x;
  if (a >= V) return;
  out[a] = make_float4(z[3 * a], z[3 * a + 1], z[3 * a + 2], 0.f);
}

}  // namespace
}  // namespace cemppi

using namespace cemppi;

extern "C" ce_status ce_mppi_dbscan_noalloc(int32_t device, const float* z, int32_t V, int32_t p,
                                            float eps, int32_t min_pts, int32_t* ncount,
                                            int32_t* label, int32_t* n_clusters, void* stream) {
  if (V < 0 || (size_t)V > kMaxPts)
    return set_error(CE_EINVAL, "V outside 0.." + std::to_string(kMaxPts) + " (the scratch capacity)");
  if (p != 2 && p != 3) return set_error(CE_EINVAL, "p must be 2 or 3");
  if (!(eps > 0.f) || !(eps < INFINITY)) return set_error(CE_EINVAL, "eps must be finite and > 0");
  if (min_pts < 1) return set_error(CE_EINVAL, "min_pts must be >= 1");
  if (V > 0 && (!z || !label)) return set_error(CE_EINVAL, "z and label must not be NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return set_error(CE_EINVAL, "device ordinal out of range");
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != device && hipSetDevice(device) != hipSuccess) return set_error(CE_EDEVICE, "hipSetDevice");
  char* base = nullptr;
  ce_status st = scratch_of(device, &base);
  if (st == CE_OK) {
    Cfg c{};
    c.p = p;
    c.K = V;
    c.eps2 = eps * eps;
    c.min_pts = min_pts;
    c.ntile = (V + kTile - 1) / kTile;
    c.mcap = V;
    Bufs b{};
    b.ctrl = reinterpret_cast<Ctrl*>(base + o_ctrl);
    b.ncount = reinterpret_cast<int*>(base + o_ncount);
    b.mcn = reinterpret_cast<int*>(base + o_mcn);
    b.root = reinterpret_cast<int*>(base + o_root);
    b.label = reinterpret_cast<int*>(base + o_label);
    b.coremask = reinterpret_cast<unsigned long long*>(base + o_core);
    b.hookmask = reinterpret_cast<unsigned long long*>(base + o_hook);
    b.tadj = reinterpret_cast<unsigned long long*>(base + o_tadj);
    float4* pack = reinterpret_cast<float4*>(base + o_pack);
    b.gv = reinterpret_cast<float*>(pack);
    b.z = b.gv;
    Launcher L(reinterpret_cast<hipStream_t>(stream));
    const float* zin = z;
    if (V > 0 && p == 3) {
      L(k_pack3, dim3((V + 255) / 256), dim3(256), z, (int)V, pack);
      zin = b.gv;
    }
    launch_stage_dbscan(L, c, b, zin, V, ncount, label, n_clusters);
    if (L.err != hipSuccess) st = set_hip_error(L.err, "dbscan_noalloc launch");
  }
  if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
  return st;
}
