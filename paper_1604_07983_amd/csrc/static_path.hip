// static_path.hip -- the whole path for one geometry without device
// allocation, for callers that cannot allocate (code under stream capture,
// serving loops): every device buffer comes from one file-scope array.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/nbs.h"
#include "plan_internal.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)NBS_STATIC_WORKSPACE_MIB << 20;

// The workspace: each device that runs the path holds its own copy until
// the process ends.  Host code never passes this name to a kernel; it uses
// the device address looked up once per device below.
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_scratch[kMaxDevices];
char g_msg[256];

// Address of the current device's copy of the workspace, looked up on the
// device's first call.
nbs_status scratch_of(int device, void** ptr) {
  std::lock_guard<std::mutex> hold(g_lock);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      std::snprintf(g_msg, sizeof g_msg, "hipGetSymbolAddress: %s", hipGetErrorString(e));
      return NBS_ERR_DEVICE;
    }
    g_scratch[device] = p;
  }
  *ptr = g_scratch[device];
  return NBS_OK;
}

}  // namespace

extern "C" {

nbs_status nbs_four_point_static(const nbs_geometry* g, const nbs_channel* ch, int32_t n_ch, nbs_precision precision,
                                 const void* prop_u, const void* prop_d, const void* prop_s, void* F_out,
                                 void* stream) {
  std::snprintf(g_msg, sizeof g_msg, "%s", "");
  if (!g || !ch || !prop_u || !prop_d || !prop_s || !F_out) {
    std::snprintf(g_msg, sizeof g_msg, "null argument");
    return NBS_ERR_INVALID;
  }
  int device = -1;
  if (hipGetDevice(&device) != hipSuccess || device < 0 || device >= kMaxDevices) {
    std::snprintf(g_msg, sizeof g_msg, "no current device");
    return NBS_ERR_DEVICE;
  }
  void* base = nullptr;
  nbs_status s = scratch_of(device, &base);
  if (s != NBS_OK) return s;
  nbs_plan p = nullptr;
  hipStream_t st = (hipStream_t)stream;
  s = nbs::create_plan(&p, g, 1, ch, n_ch, precision, device, base, kScratchBytes, st);
  if (s != NBS_OK) {
    const char* why = p ? nbs::plan_error(p) : nbs::create_error();
    std::snprintf(g_msg, sizeof g_msg, "%s", why[0] ? why : "invalid geometry, channels or precision");
    if (p) nbs_plan_destroy(p);
    return s;
  }
  const void* pu[1] = {prop_u};
  const void* pd[1] = {prop_d};
  const void* ps[1] = {prop_s};
  void* fo[1] = {F_out};
  s = nbs::run_plan(p, pu, pd, ps, fo, st);
  if (s != NBS_OK) std::snprintf(g_msg, sizeof g_msg, "%s", nbs::plan_error(p));
  nbs_plan_destroy(p);
  return s;
}

const char* nbs_static_last_error(void) { return g_msg; }

}  // extern "C"
