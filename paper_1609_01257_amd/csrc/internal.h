// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "rngx.h"

namespace rngx {

// ---- errors ---------------------------------------------------------------
// Record a message for the calling thread and return `code`.
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int hip_fail(hipError_t e, const char *what);
void clear_error();

#define RNGX_HIP(call)                                   \
    do {                                                 \
        hipError_t rngx_e_ = (call);                     \
        if (rngx_e_ != hipSuccess)                       \
            return ::rngx::hip_fail(rngx_e_, #call);     \
    } while (0)

// ---- the two hashes of the init kernel (host copies, used to fold the seed)
// Listing S4, "low bits": six-round 32-bit integer hash.
__host__ __device__ __forceinline__ uint32_t hash_low(uint32_t a)
{
    a = (a + 0x7ed55d16u) + (a << 12);
    a = (a ^ 0xc761c23cu) ^ (a >> 19);
    a = (a + 0x165667b1u) + (a << 5);
    a = (a + 0xd3a2646cu) ^ (a << 9);
    a = (a + 0xfd7046c5u) + (a << 3);
    a = (a ^ 0xb55a4f09u) ^ (a >> 16);
    return a;
}

// Listing S4, "high bits": five-round shift-multiply hash.
__host__ __device__ __forceinline__ uint32_t hash_high(uint32_t a)
{
    a = (a ^ 61u) ^ (a >> 16);
    a = a + (a << 3);
    a = a ^ (a >> 4);
    a = a * 0x27d4eb2du;
    a = a ^ (a >> 15);
    return a;
}

// Listing S5: one step of the (21,35,4) xorshift.
__host__ __device__ __forceinline__ uint64_t xs_step(uint64_t x)
{
    x ^= x << 21;
    x ^= x >> 35;
    x ^= x << 4;
    return x;
}

// Seed folded into the two hash inputs: low = J(gid ^ mix_low),
// high = W(low ^ mix_high); both are 0 for seed 0 (the paper's init).
struct SeedMix {
    uint32_t mix_low;
    uint32_t mix_high;
    uint32_t zero_fix; // W(0): high word of the replacement for a zero state
};

inline SeedMix seed_mix(uint64_t seed)
{
    SeedMix m;
    m.mix_low = hash_low((uint32_t)seed) ^ hash_low(0u);
    m.mix_high = hash_high((uint32_t)(seed >> 32)) ^ hash_high(0u);
    m.zero_fix = hash_high(0u);
    return m;
}

__host__ __device__ __forceinline__ uint64_t init_state(const SeedMix &m, uint32_t gid)
{
    uint32_t lo = hash_low(gid ^ m.mix_low);
    uint32_t hi = hash_high(lo ^ m.mix_high);
    uint64_t x = ((uint64_t)hi << 32) | lo;
    return x != 0u ? x : ((uint64_t)m.zero_fix << 32);
}

// ---- kernel launchers (kernels.hip) ---------------------------------------
hipError_t launch_init(uint64_t *state, uint32_t n, const SeedMix &mix, hipStream_t s);
hipError_t launch_gen(const rngx_launch &cfg, bool u32, uint64_t *state, uint32_t n,
                      uint32_t iters, void *out, hipStream_t s);
bool launch_cfg_valid(const rngx_launch &cfg);

// ---- the process-wide generator context (api.cpp) --------------------------
struct Generator {
    std::recursive_mutex mu; // re-entrant: a stream consumer may call back in
    bool inited = false;
    int device = -1;
    uint64_t seed = 0;
    uint32_t n = 0;
    uint64_t cursor = 0;
    uint64_t *state = nullptr;       // n states, library-owned device memory
    hipStream_t lib_stream = nullptr; // the init kernel's stream
    hipEvent_t state_ready = nullptr; // last use of `state` (any stream)
    rngx_launch cfg64{512, 4, 0}; // fastest measured at 2^26 x 256 on MI355X
    rngx_launch cfg32{512, 2, 0};
    // Streams and events of the device-to-host pipeline (pipeline.cpp).
    hipStream_t pipe_gen = nullptr, pipe_copy = nullptr;
    hipEvent_t gen_done[2] = {nullptr, nullptr};
    hipEvent_t copy_done[2] = {nullptr, nullptr};
};

Generator &generator();
// Enqueue n_iters iterations into `out` on stream `s`; caller holds g.mu.
int generate_locked(Generator &g, uint32_t n_iters, void *out, hipStream_t s, bool u32);
int check_device_locked(const Generator &g);
void release_pipeline_locked(Generator &g);

// ---- profiler (profiler.cpp) ----------------------------------------------
namespace prof {
// Open a timed operation on `s`: records its start event. Returns a token
// (or -1 when logging is off or the log is full).
int begin(const char *name, hipStream_t s);
// Close it: records its end event on the same stream.
void end(int token, hipStream_t s);
// Restart the window (log cleared, host clock and reference event reset).
int start(hipStream_t ref_stream);
int stop();
void release_all();
int stats(rngx_prof_stats *out);
const char *summary();
int events(rngx_prof_event *out, uint32_t cap, uint32_t *n_out);
int enable(int on);
} // namespace prof
int analyze_table(const rngx_prof_event *events, uint32_t n, double elapsed_s,
                  rngx_prof_stats *out);

} // namespace rngx
