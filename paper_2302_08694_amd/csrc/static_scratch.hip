// Type-1 transform for callers that cannot allocate device memory (fsib_spread_noalloc).
//
// Every per-call buffer of the transform -- the point sort (bins, ranks, sorted records), the spreading
// work list and partial tiles, the fine grid and the FFT intermediates -- is carved from one static
// device array instead of the plan's workspace, so the call makes no hipMalloc, hipFree or other
// allocating call, and its point count is bounded by the array rather than by the plan's max_points.
// The array lives in the code object: each GPU the library runs on holds its own copy, at its own
// address, until the process ends.  Host code never uses the array's name as a device address (on
// the host it names a stand-in); the device address is looked up once per device with
// hipGetSymbolAddress and kept.
#include <mutex>

#include "plan.hpp"

namespace {

constexpr int64_t kScratchBytes = FSIB_NOALLOC_SCRATCH_BYTES;  // per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of the static array on `device` (current), looked up on the first call there.
fsib_status scratch_on(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fsib::report(FSIB_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fsib::report(FSIB_ERR_HIP, (std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)).c_str());
    }
    g_scratch[device] = ptr;
  }
  *out = g_scratch[device];
  return FSIB_OK;
}

}  // namespace

extern "C" fsib_status fsib_spread_noalloc(fsib_plan plan, int64_t M, const double* X, const void* c, void* fhat,
                                           double scale, void* stream) {
  int device = -1;
  const hipError_t e = hipGetDevice(&device);
  if (e != hipSuccess) return fsib::report(FSIB_ERR_HIP, (std::string("hipGetDevice: ") + hipGetErrorString(e)).c_str());
  void* ws = nullptr;
  const fsib_status s = scratch_on(device, &ws);
  if (s != FSIB_OK) return s;
  return fsib::spread_in_workspace(plan, device, M, X, c, fhat, scale, stream, ws, kScratchBytes);
}
