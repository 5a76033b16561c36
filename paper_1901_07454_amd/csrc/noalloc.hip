// noalloc.hip -- arb_get_voltages_noalloc: voltages to host memory without
// allocating device memory.
//
// arb_get_voltages with a host destination gathers the packed voltages into
// user CV order in a device staging buffer the sim allocates on its first
// such call.  This variant stages through a fixed array of static device
// memory instead (scratch, kNoallocDoubles doubles = 64 MiB; every GPU the
// library runs on holds its own copy until the process ends), for callers
// that cannot allocate.  Host code never passes the array's name to a
// kernel or a copy: its device address is taken once per device, at sim
// set-up, with hipGetSymbolAddress, and that pointer is used.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "../../include/arbmi.h"
#include "kernels.hpp"
#include "sim.hpp"

namespace arbmi {

constexpr int64_t kNoallocDoubles = int64_t(1) << 23;  // 64 MiB of staging

static __device__ __align__(256) double scratch[kNoallocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};      // scratch's device address on each device
hipError_t g_status[kMaxDevices] = {}; // result of the lookup (hipSuccess once found)
bool g_tried[kMaxDevices] = {};

}  // namespace

// Once per device, with that device current: the address of its scratch.
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_tried[device]) return g_status[device];
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_tried[device] = true;
    g_status[device] = e;
    if (e == hipSuccess) g_ptr[device] = static_cast<double*>(ptr);
    return e;
}

}  // namespace arbmi

using namespace arbmi;

extern "C" int arb_get_voltages_noalloc(arb_sim s_, double* dst, int64_t n) {
    Sim* s = static_cast<Sim*>(s_);
    if (!s || !dst) return set_error(ARB_EINVAL, "null argument");
    const int64_t ncv = s->L.n_cv;
    if (n < ncv) return set_error(ARB_EINVAL, "destination smaller than the CV count");
    if (ncv > kNoallocDoubles) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "the model has %lld CVs, more than the %lld the static staging buffer holds",
                      (long long)ncv, (long long)kNoallocDoubles);
        return set_error(ARB_EINVAL, msg);
    }
    double* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        if (s->device >= 0 && s->device < kMaxDevices && g_tried[s->device] && g_status[s->device] == hipSuccess)
            ptr = g_ptr[s->device];
    }
    if (!ptr) return set_error(ARB_EHIP, "static staging buffer unavailable on the sim's device");
    hipError_t e = launch_gather(s->d_V, s->d_perm, ptr, ncv, s->st);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, ptr, size_t(ncv) * 8, hipMemcpyDeviceToHost, s->st);
    if (e == hipSuccess) e = hipStreamSynchronize(s->st);
    if (e != hipSuccess) return set_hip_error(e, "arb_get_voltages_noalloc");
    return ARB_OK;
}
