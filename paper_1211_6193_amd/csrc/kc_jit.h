// Program-specialised free-run and replay kernels (host side).
#pragma once
#include <memory>
#include <string>

#include "kc_internal.h"

namespace kc {

struct JitEntry;
struct JitFunctions {
    hipFunction_t local_256 = nullptr;    // epoch-local check, workgroups up to 256 threads
    hipFunction_t local_1024 = nullptr;   // epoch-local check, up to 1024 threads
    hipFunction_t free_1024 = nullptr;    // every access logged
    hipFunction_t lock_local = nullptr;   // lockstep replay, epoch-local check
    hipFunction_t lock_local_256 = nullptr;   // ... workgroups up to 256 threads (no register bound)
    hipFunction_t lock = nullptr;         // lockstep replay, every access logged
};

// HIP source of the specialised kernels of a program (validated words);
// `waves` > 0 asks the compiler for that many waves per SIMD.
std::string jit_source(const uint64_t *words, uint32_t n, int waves);
// Cache entry of (program, waves) (created uncompiled).
std::shared_ptr<JitEntry> jit_request(const uint64_t *words, uint32_t n, int waves);
// true if the caller took the job of compiling the entry (it was uncompiled).
bool jit_claim(const std::shared_ptr<JitEntry> &e);
// Compile a claimed entry (CPU only, hiprtc); waiters on the entry are woken.
void jit_compile(const std::shared_ptr<JitEntry> &e);
// The kernels on `device` (the current device), loading the module on first
// use.  false if the entry is not compiled, is being compiled by another
// thread (unless `wait`) or failed.
bool jit_functions(const std::shared_ptr<JitEntry> &e, int device, bool wait, JitFunctions &out,
                   double *compile_ms);
int jit_state(const std::shared_ptr<JitEntry> &e);       // 0 uncompiled, 2 compiling, 1 ready, -1 failed
std::string jit_log(const std::shared_ptr<JitEntry> &e);
// Whether the free-run LDS layout of such a launch fits the 64 KiB a module
// kernel may take, and the launch itself (same arguments as launch_interp).
bool jit_fits(uint32_t sh_words_max, uint32_t wg_threads);
hipError_t launch_jit(const JitFunctions &f, const InterpArgs &a, uint32_t n_wg, uint32_t wg_threads,
                      hipStream_t s);
// A lockstep replay launch of one program's components (same arguments as
// launch_interp with lockstep set); hipErrorInvalidValue if it does not fit.
hipError_t launch_jit_lockstep(const JitFunctions &f, const InterpArgs &a, uint32_t n_wg, uint32_t wg_threads,
                               hipStream_t s);

}  // namespace kc
