// Entry points that allocate nothing, for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid it).  Their scratch is one fixed array of the
// library in device memory; each device holds its own copy at its own
// address, found once per device with hipGetSymbolAddress and used by
// address from then on (the array's name is not a device address on the
// host).
#include <mutex>

#include "runtime_int.h"

using namespace mgrt;

namespace {

// Block partial sums of a prefix sum of up to NOALLOC_SCAN_MAX elements:
// 2^31 / 2048 + 2^31 / 2048^2 sums of 8 bytes, plus a little (8.4 MB).
constexpr int64_t NOALLOC_SCAN_MAX = (int64_t)1 << 31;
constexpr size_t NOALLOC_BYTES = (size_t)17 << 19;  // 8.5 MiB

__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

}  // namespace

namespace mgrt {

// Device address of this device's scratch array (device current), looked up
// once per device.
hipError_t noalloc_scratch(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

}  // namespace mgrt

extern "C" {

magnus_status_t magnus_exclusive_scan_i64_noalloc(magnus_handle_t h, const int64_t* in,
                                                  int64_t* out, int64_t n, int64_t* total,
                                                  void* stream) {
  if (!h || n < 0 || (n > 0 && (!in || !out))) return MAGNUS_ERR_INVALID_ARG;
  if (n > NOALLOC_SCAN_MAX || scan_temp_bytes(n) > NOALLOC_BYTES) {
    h->err = "more elements than the fixed scratch holds (2^31)";
    return MAGNUS_ERR_WORKSPACE;
  }
  HIPCHK(hipSetDevice(h->device));
  void* tmp = nullptr;
  HIPCHK(noalloc_scratch(h->device, &tmp));
  HIPCHK(scan_excl_i64(in, out, n, total, nullptr, tmp, (hipStream_t)stream));
  return MAGNUS_OK;
}

}  // extern "C"
