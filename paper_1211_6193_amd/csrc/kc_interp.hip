// Interpreter kernels (free run with and without the epoch-local check, and
// the lockstep replay) and their host launchers; the device code is in
// kc_device.h.
#include "kc_device.h"

#include <mutex>

namespace kc {

namespace {

// Free-run kernels: with the epoch-local check (shadow tuples and local sort)
// and without it; occupancy targets keep them free of register spills.
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5, 5))) k_interp_free_local(InterpArgs A) {
    interp_free_body<true>(A);
}
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(6, 6))) k_interp_free(InterpArgs A) {
    interp_free_body<false>(A);
}

__global__ void __launch_bounds__(1024) k_interp_lockstep(InterpArgs A) { interp_lockstep_body<false>(A); }
__global__ void __launch_bounds__(1024) k_interp_lockstep_local(InterpArgs A) { interp_lockstep_body<true>(A); }
__global__ void __launch_bounds__(1024) k_interp_lockstep_sites(InterpArgs A) { interp_lockstep_sites_body(A); }

}  // namespace

// Raise the dynamic LDS limit of the interpreter kernels to 160 KiB, once per
// device: batch worker threads may launch for the first time together.
static hipError_t raise_lds_limits() {
    constexpr int kMaxDevices = 64;
    static std::once_flag once[kMaxDevices];
    static hipError_t result[kMaxDevices];
    int dev = 0;
    const hipError_t eg = hipGetDevice(&dev);
    if (eg != hipSuccess) return eg;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(once[dev], [dev] {
        const void *kernels[] = {(const void *)k_interp_free, (const void *)k_interp_free_local,
                                 (const void *)k_interp_lockstep, (const void *)k_interp_lockstep_local,
                                 (const void *)k_interp_lockstep_sites};
        hipError_t e = hipSuccess;
        for (const void *k : kernels) {
            const hipError_t ek = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (e == hipSuccess) e = ek;
        }
        result[dev] = e;
    });
    return result[dev];
}

uint32_t gst_bits_for(uint32_t wg_threads) {
    uint32_t b = 8;
    while ((1u << b) < 4u * wg_threads) b++;
    return b;
}

size_t interp_lds_bytes(uint32_t sh_words_max, uint32_t wg_threads, uint32_t stage, bool lockstep, bool local,
                        uint32_t gst_bits) {
    const uint32_t nwaves = (wg_threads + WAVE - 1) / WAVE;
    size_t off = ((size_t)sh_words_max * 4 + 15) & ~(size_t)15;
    off += (size_t)nwaves * stage * 8;
    if (local) off += (size_t)nwaves * stage * 8 + (size_t)nwaves * 256 * 4 + 256 * 4 + shadow_region_bytes(sh_words_max);
    if (local && gst_bits) off += ((size_t)8 << gst_bits) + (size_t)rep_hold_for(wg_threads) * 8;
    off += (16 * 10 + 16 * 4 + 3 * 8) * 4 + (size_t)(sh_words_max + 31) / 32 * 4;
    if (lockstep) off += (size_t)sh_words_max * 4 + ((size_t)8 << lockstep_hash_bits(wg_threads));
    return off;
}

hipError_t launch_interp(const InterpArgs &a, uint32_t n_wg, uint32_t wg_threads, bool lockstep, hipStream_t s) {
    if (n_wg == 0) return hipSuccess;
    InterpArgs args = a;
    args.rep_hold = rep_hold_for(wg_threads);
    if (args.sites) args.local = 0;                   // the source-site replay logs every access
    if (!args.local) args.gst_bits = 0;
    auto bytes = [&] {
        return interp_lds_bytes(args.sh_words_max, wg_threads, args.stage, lockstep, args.local != 0, args.gst_bits);
    };
    size_t lds = bytes();
    while (lds > 160 * 1024 && args.stage > 64) {   // shrink the record staging area to fit
        args.stage = (args.stage / 2 + 63) / 64 * 64;
        lds = bytes();
    }
    if (lds > 160 * 1024 && args.gst_bits) {          // no room for the table: stage and sort
        args.gst_bits = 0;
        lds = bytes();
    }
    if (lds > 160 * 1024 && args.local) {             // no room for the epoch-local check: log everything
        args.local = 0;
        lds = bytes();
    }
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const hipError_t ea = raise_lds_limits();
    if (ea != hipSuccess) return ea;
    if (lockstep && args.sites)
        hipLaunchKernelGGL(k_interp_lockstep_sites, dim3(n_wg), dim3(wg_threads), lds, s, args);
    else if (lockstep && args.local)
        hipLaunchKernelGGL(k_interp_lockstep_local, dim3(n_wg), dim3(wg_threads), lds, s, args);
    else if (lockstep)
        hipLaunchKernelGGL(k_interp_lockstep, dim3(n_wg), dim3(wg_threads), lds, s, args);
    else if (args.local)
        hipLaunchKernelGGL(k_interp_free_local, dim3(n_wg), dim3(wg_threads), lds, s, args);
    else
        hipLaunchKernelGGL(k_interp_free, dim3(n_wg), dim3(wg_threads), lds, s, args);
    return hipGetLastError();
}

}  // namespace kc
