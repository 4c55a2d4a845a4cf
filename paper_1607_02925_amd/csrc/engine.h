// Internal interface between the solve engine and the request server.  Not
// part of the C ABI: nothing here crosses the library boundary.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "lowrank.h"

struct lr_plan_s;

namespace lr {

// Pinned host staging buffer of a plan: holds the largest device-to-host read
// of the solve loop (two 64 x 64 FP64 blocks).
constexpr size_t HOST_PIN_BYTES = 64 * 64 * sizeof(double) * 2;

// Host-side resources a plan borrows instead of creating its own: the pinned
// staging buffer (HOST_PIN_BYTES) and eight timing events.
struct HostRes {
  double* hpin;
  hipEvent_t ev[8];
};

void set_last_error(const std::string& msg);
std::string last_error();

// Argument checks of lowrank_plan (sets the thread's error message).
lr_status plan_check(const lr_matrix* X, int k, int p, double eps, const lr_options* opt);
// Device workspace bytes a plan for X, k, p needs.
lr_status plan_bytes(const lr_matrix* X, int k, int p, const lr_options* opt, size_t* bytes);
// Build a plan on stream `st`.  ws == nullptr: the plan allocates and owns its
// workspace; otherwise its buffers are carved from ws (ws_bytes >= plan_bytes)
// and ws stays the caller's.  host == nullptr: the plan creates its own pinned
// buffer and events; otherwise it borrows them.
lr_status plan_make(lr_plan_s** out, const lr_matrix* X, int k, int p, double eps,
                    const lr_options* opt, hipStream_t st, void* ws, size_t ws_bytes,
                    const HostRes* host);
// Plan on the stack with a borrowed workspace (ws_bytes >= plan_bytes) and
// borrowed host resources, one lowrank_solve, nothing kept.  Dense X only;
// opt->timing must be 0 (host->ev may be null).
lr_status solve_borrowed(const lr_matrix* X, int k, int p, double eps, const lr_options* opt,
                         hipStream_t st, void* ws, size_t ws_bytes, const HostRes* host,
                         double* U_out, double* theta_out, lr_report* rep);
lr_status host_res_create(double** hpin, hipEvent_t* ev);
void host_res_destroy(double* hpin, hipEvent_t* ev);

}  // namespace lr
