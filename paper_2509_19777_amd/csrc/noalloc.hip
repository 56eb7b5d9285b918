// Allocation-free application of the preconditioner.
//
// hplmm_apply_noalloc runs the same kernels as hplmm_apply, but the one
// scratch buffer of the application -- the partial sums of the coarse
// sweeps' split rows -- lives in a fixed-size static device array instead of
// memory that hplmm_plan allocated.  Nothing in the call
// allocates (no hipMalloc, no events, no library routine that allocates), so
// it can run under HIP graph capture or in loops that must not allocate.
//
// Every device the library runs on holds its own copy of the array (its
// address differs per device) until the process ends; host code never passes
// the array's name to a kernel, only the address hipGetSymbolAddress returned
// for the current device.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "handle.h"

namespace hplmm {

namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;   // 8 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

void *static_scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) fail(HPLMM_E_ARG, "device index outside the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(HPLMM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace hplmm

using namespace hplmm;

extern "C" hplmm_status hplmm_apply_noalloc(hplmm_handle *hh, int32_t which, const double *r, double *z,
                                            void *stream) {
    return guarded([&]() -> hplmm_status {
        if (!hh || !r || !z) fail(HPLMM_E_ARG, "NULL argument");
        if (r == z) fail(HPLMM_E_ARG, "r and z must not alias");
        if (which < 0 || which > 4) fail(HPLMM_E_ARG, "which must be 0..4");
        Handle &h = hh->h;
        if (!h.ready) fail(HPLMM_E_STATE, "hplmm_setup has not completed");
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) fail(HPLMM_E_HIP, "hipGetDevice failed");
        if (cur != h.device) fail(HPLMM_E_ARG, "the handle's device is not the current device");
        // the split-row partial sums (doubles); every one is written by its
        // chunk before the reduction launch reads it, so nothing needs clearing
        const size_t need = sizeof(double) * (size_t)h.gemv_part_len;
        if (need > kScratchBytes)
            fail(HPLMM_E_ARG, "the coarse sweeps need " + std::to_string(need) +
                                  " bytes of split-row scratch; the static buffer holds " +
                                  std::to_string(kScratchBytes));
        char *base = (char *)static_scratch_address(cur);
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        // route the split rows to the static buffer and keep the profiler
        // (which creates events) off for the duration of the call
        struct Restore {
            Handle &h;
            int32_t mask;
            ~Restore() {
                h.split_part = nullptr;
                h.prof.mask = mask;
            }
        } restore{h, h.prof.mask};
        h.split_part = (double *)base;
        h.prof.mask = 0;
        apply_op(h, which, r, z, s);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) fail(HPLMM_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
        return HPLMM_OK;
    });
}
