// lowrank_solve_noalloc: the whole solve with its device workspace taken from a
// fixed array in the library's device image instead of hipMalloc, for callers
// that cannot allocate device memory.
//
// The array is a file-scope __device__ symbol.  Its host-side name is only a
// stand-in for the device object, so host code never passes it to a kernel or
// a copy: the first call on each device (with that device current) looks up
// the array's device address with hipGetSymbolAddress and keeps it; every
// later use goes through that address.  Each device holds its own copy of the
// array until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "engine.h"
#include "lowrank.h"

namespace {

static __device__ __align__(256) unsigned char scratch[LR_NOALLOC_MAX_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of this device's copy of the array (looked up once).
lr_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    (void)hipGetLastError();
    lr::set_last_error("no usable current device");
    return LR_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      lr::set_last_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return LR_EDEVICE;
    }
    g_scratch[dev] = ptr;
  }
  *out = g_scratch[dev];
  return LR_OK;
}

// Host staging for the solve loop's small device-to-host reads, one per
// calling thread (pageable: the copies into it are synchronous anyway).
thread_local double t_stage[lr::HOST_PIN_BYTES / sizeof(double)];

}  // namespace

extern "C" lr_status lowrank_solve_noalloc(const lr_matrix* X, int k, int p, double eps,
                                           const lr_options* opt, void* hip_stream,
                                           double* U_out, double* theta_out, lr_report* rep) {
  size_t need = 0;
  lr_status s = lr::plan_bytes(X, k, p, opt, &need);
  if (s != LR_OK) return s;
  if (need > (size_t)LR_NOALLOC_MAX_BYTES) {
    lr::set_last_error("the problem needs " + std::to_string(need) +
                       " bytes of device workspace; lowrank_solve_noalloc holds " +
                       std::to_string((size_t)LR_NOALLOC_MAX_BYTES));
    return LR_ENOMEM;
  }
  void* ws = nullptr;
  s = scratch_address(&ws);
  if (s != LR_OK) return s;
  lr::HostRes host{};
  host.hpin = t_stage;
  return lr::solve_borrowed(X, k, p, eps, opt, (hipStream_t)hip_stream, ws, need, &host, U_out,
                            theta_out, rep);
}
