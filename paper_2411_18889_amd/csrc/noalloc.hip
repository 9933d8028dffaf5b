// nbody_accel_noalloc: nbody_accel for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation). The pass and its kernels are nbody_accel's; only the
// scratch differs: a fixed-size device array of this file instead of the
// caller's workspace.
#include <mutex>

#include "common.h"

namespace {

using namespace nb;

// The scratch: a file-scope device array of NB_NOALLOC_SCRATCH_BYTES. Every
// device the library runs on holds its own copy from the time the library's
// code is loaded there until the process ends. In host code its name is not
// a device address: the address of each device's copy is taken once, with
// that device current, and kept; every launch gets that address.
constexpr size_t kScratchBytes = size_t(NB_NOALLOC_SCRATCH_BYTES);
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch, set up on the first
// call on that device.
int scratch_address(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices) return NB_ENODEV;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        if (!p) return NB_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return NB_OK;
}

}  // namespace

extern "C" int nbody_accel_noalloc(int64_t ni, const void* xi, int64_t nj, const void* xj,
                                   const void* mj, double eps, double G, int prec, void* acc,
                                   void* pot, void* stream) {
    AccelPlan plan;
    int st = accel_plan(ni, xi, nj, xj, mj, eps, G, prec, acc, pot, nullptr, &plan);
    if (st != NB_OK) return st;
    if (plan.need > kScratchBytes) return NB_EWORKSPACE;
    if ((st = check_device()) != NB_OK) return st;
    // every pass writes each scratch element it reads back before reading it,
    // so nothing has to be cleared between calls
    void* ws = nullptr;
    if (plan.need > 0 && (st = scratch_address(&ws)) != NB_OK) return st;
    return hip_status(accel_launch(plan, ni, xi, nj, xj, mj, eps, G, prec, acc, pot, ws,
                                   std::min(kScratchBytes, plan.full),
                                   static_cast<hipStream_t>(stream)));
}
