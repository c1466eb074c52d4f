// Host-side services of the ray-tracing library that the serving layer
// (frt_server.cpp) takes beside the public C ABI of include/frt.h.  Nothing
// here names a HIP type, so the serving layer also builds against another
// implementation of these calls and of the ABI (a CPU stand-in for the
// scheduler's tests).
#pragma once
#include <cstddef>
#include <cstdint>

#include "frt.h"

// Solves one launch sequence steps together (and the server's slot limit).
#define FRT_MAX_SOLVES_PER_LAUNCH 1024

namespace frt {
// Set the calling thread's error message (returned by frt_last_error) and
// return code.
int set_error(int code, const char* msg);
int ctx_device(frt_ctx ctx);
// Device bytes a solve with these parameters and sizes holds, and the first
// pass-queue size it asks for (records, and their bytes, which are part of
// the total: the pass queues are shared by the solves of a context and grow
// with the largest pass).
uint64_t solve_bytes(const frt_params& P, uint64_t ncell, int n_src, int with_T, uint64_t* pass_records,
                     uint64_t* pass_bytes);
// Device bytes the context's shared pass queues hold now, and the most they
// may grow to (0: no limit; a step that needs more fails with FRT_ENOMEM
// before anything runs).  Trimming frees them (the next step allocates them
// again at its own size); only while no step of the context is running.
uint64_t ctx_workspace_bytes(frt_ctx ctx);
void ctx_set_workspace_limit(frt_ctx ctx, uint64_t bytes);
void ctx_trim_workspace(frt_ctx ctx);
// Make `device` the calling thread's device (threads the layer starts).
int use_device(int device);
// Copy `bytes` from device memory to host memory after all work queued on
// the device has finished.
int copy_device_to_host(void* dst, const void* src, size_t bytes);
// Seconds on a monotonic clock; request times are differences of it.
double clock_s();
}  // namespace frt
