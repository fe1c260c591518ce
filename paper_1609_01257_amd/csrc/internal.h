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

// ---- batched streams (batch.hip, batch.cpp) -------------------------------
// One request as the batch kernel reads it (64 bytes). Requests of length 0
// are dropped on the host. The seed is folded in already (SeedMix fields).
// Tiles are laid over a virtual index space in which the request occupies
// [vbase, vbase + length); value t of the request is stored at dst[t].
struct BatchReq {
    uint64_t offset;     // value number of the request's first value
    uint64_t length;     // values requested (> 0)
    uint64_t vbase;      // first virtual index (tiling only)
    uint64_t item_begin; // number of the request's first work item
    uint64_t first_tile; // first tile (of C = 64 * S values) it touches
    uint32_t gid;
    uint32_t mix_low;
    uint32_t mix_high;
    uint32_t zero_fix;
    uint64_t *dst;       // destination of value 0 (16-byte alignment of
                         // dst - vbase, i.e. dst aligned as vbase is even)
};
static_assert(sizeof(BatchReq) == 64, "BatchReq layout");

// Fill one request record for tiles of C values; returns the number of work
// items (tiles) the request touches.
inline uint64_t make_record(BatchReq &r, uint64_t offset, uint64_t length, uint64_t vbase,
                            uint64_t item_begin, uint32_t gid, const SeedMix &mix, uint64_t *dst,
                            uint64_t C)
{
    r.offset = offset;
    r.length = length;
    r.vbase = vbase;
    r.item_begin = item_begin;
    r.first_tile = vbase / C;
    r.gid = gid;
    r.mix_low = mix.mix_low;
    r.mix_high = mix.mix_high;
    r.zero_fix = mix.zero_fix;
    r.dst = dst;
    return (vbase + length - 1) / C - r.first_tile + 1;
}

// Launch descriptor, read by the kernel from device memory so a captured
// graph can be replayed with new contents. With `states` set, a request's
// stream starts from states[gid] (resident states) instead of H(seed, gid).
// `next_item` is the work counter the waves take items from; it is 0 in the
// staged copy, so every upload of the table (also a graph replay) resets it.
struct BatchDesc {
    const BatchReq *reqs;
    const uint64_t *states;
    uint64_t n_items;
    uint32_t m;
    uint32_t reserved0;
    uint64_t next_item;
    uint64_t reserved1[3];
};
static_assert(sizeof(BatchDesc) == 64, "BatchDesc layout");
// Offset of the request records in a staged or device table. The records
// start one 128-byte L2 line after the descriptor, so that no record shares
// a line with the work counter, which every wave of a persistent launch
// updates atomically.
constexpr size_t kReqOffset = 128;
static_assert(kReqOffset >= sizeof(BatchDesc) && kReqOffset % 64 == 0, "request offset");

// A batch of at most kSmallReqs requests travels in the kernel's arguments
// (1,088 bytes) instead of being uploaded: one launch, no copy before it.
constexpr uint32_t kSmallReqs = 16;
struct SmallTable {
    BatchDesc desc;
    BatchReq reqs[kSmallReqs];
};

// A staging/upload slot for one batch in flight (batch.cpp).
struct BatchSlot {
    int device = -1;          // the device its buffers, event and graph are on
    uint32_t capacity = 0;    // requests the buffers hold (power of two)
    void *staging = nullptr;  // page-locked: BatchDesc, then capacity BatchReq at kReqOffset
    void *devtab = nullptr;   // device copy of the same
    hipEvent_t done = nullptr; // recorded after the slot's last launch
    hipGraphExec_t exec = nullptr;
    rngx_batch_cfg exec_cfg{};
    bool exec_star = false;
    hipStream_t cap_stream = nullptr;
    uint32_t m_staged = 0;
    uint64_t n_items = 0;
};

bool batch_cfg_valid(const rngx_batch_cfg &c);
// Index of an allowed values-per-lane S in the per-S tables.
int batch_s_index(uint32_t s);
// Index of an allowed group size of the grouped order, or -1.
int batch_group_index(uint32_t g);
// Blocks of the grouped kernel that fit on one compute unit at once.
hipError_t batch_group_occupancy(const rngx_batch_cfg &c, int *blocks_per_cu);
// Entries of the per-S carry table: 16 nibble positions x 16 values.
constexpr int kCarryTable = 256;
// Entries of the per-S lane-spread table: 16 nibble positions x 16 values x
// 64 lanes (128 KiB).
constexpr int kSpreadTable = 16 * 16 * 64;
// Device tables one batch launch needs, for its values-per-lane S.
struct BatchTables {
    const uint64_t *pow2;       // T^(2^b), b < 64: 64 rows each
    const uint64_t *spread;     // T^(m S) (v << 4q) at ((16 q + v) * 64 + m)
    const uint64_t *carry_nib; // T^(63 S) (next tile, same lane) as kCarryTable nibble entries
    const uint64_t *group_nib; // grouped order: T^(g 64 S - S) (tile g on), or null
    uint32_t clock_khz;        // rate of the constant-rate clock
};
// Device copies of the jump tables for the current device (thread-safe).
int batch_tables_locked(const uint64_t **pow2, const uint64_t **spread_all, int *n_cus,
                        const uint64_t **carry_nib_all = nullptr,
                        const uint64_t **group_nib_all = nullptr, int *clock_khz = nullptr);
// The configuration a launch runs: blocks 0 resolved (8 waves per compute
// unit), or for the grouped order every block that fits, in whole groups.
int resolve_batch_cfg(const rngx_batch_cfg &c, int n_cus, rngx_batch_cfg *out);
// The tables of one launch's S (and group size) among the per-device ones.
void fill_batch_tables(BatchTables &t, const rngx_batch_cfg &cfg, const uint64_t *pow2,
                       const uint64_t *spread_all, const uint64_t *nib_all,
                       const uint64_t *group_all, int clock_khz);
// Argument checks of a batched call; *total_out = the values requested.
int batch_validate(const rngx_req *reqs, uint32_t m, const uint64_t *out, uint64_t out_cap,
                   uint64_t *total_out);
int batch_stage(BatchSlot &slot, const rngx_req *reqs, uint32_t m, uint64_t *out,
                uint64_t out_cap, uint32_t values_per_lane, uint64_t *total_out);
// One request as staged by a host-side producer (the batch API or the server).
struct StageReq {
    uint64_t offset;
    uint64_t length; // > 0
    uint64_t vbase;
    uint64_t *dst;
    uint32_t gid;
    SeedMix mix;
};
int batch_stage_items(BatchSlot &slot, const StageReq *items, uint32_t k,
                      uint32_t values_per_lane, const uint64_t *states);
// star: emit the scrambled words. fit_grid: shrink the persistent grid to the
// staged work (direct launches).
int batch_launch(BatchSlot &slot, const rngx_batch_cfg &cfg, bool star, hipStream_t stream,
                 bool fit_grid = false, const char *prof_name = "BATCH_KERNEL");
// The output scrambler set by rngx_set_scrambler (api.cpp; lock-free read).
int current_scrambler();
void release_slot(BatchSlot &slot);
void release_batch();
// The batch API's launch configuration (rngx_set_batch_cfg / the autotuner).
rngx_batch_cfg current_batch_cfg();
void release_server(); // serve.cpp: stop the server, free its resources
int checksum_locked(const uint64_t *data, uint64_t n, hipStream_t s, uint64_t *result);
hipError_t launch_batch(const rngx_batch_cfg &cfg, const BatchDesc *desc, const BatchTables &t,
                        bool star, hipStream_t s);
hipError_t launch_batch_small(const rngx_batch_cfg &cfg, const SmallTable &tab,
                              const BatchTables &t, bool star, hipStream_t s);
// Checksum sum_i data[i] * (2 i + 1) mod 2^64 into *acc (device, pre-zeroed).
hipError_t launch_checksum(const uint64_t *data, uint64_t n, uint64_t *acc, hipStream_t s);

// tune.cpp: record the batched autotuner's choice in the cache named by
// RNGX_TUNE_CACHE (no-op without it); apply that cache (once, at init).
int tune_cache_record_batch(const rngx_batch_cfg &cfg, double ms, uint32_t m, uint64_t values);
int tune_cache_apply_env();

// jump.cpp: host GF(2) tables (64 matrices T^(2^b), 64 rows each).
const uint64_t *jump_tables();
uint64_t jump_host(uint64_t x, uint64_t k);
void power_rows(uint64_t k, uint64_t *rows_out);

// HIP errors with no caller to return them to (rngx_hip_notes).
// note_hip: the status of one of the library's own HIP calls on a release
// path. A failure is consumed (so that it is not reported later by an
// unrelated hipGetLastError, the library's or the application's) and
// recorded with `what`.
void note_hip(hipError_t e, const char *what);
#define RNGX_NOTE(call) ::rngx::note_hip((call), #call)
// The launchers below read a launch's status with hipGetLastError, which
// also returns an older error that no call has consumed yet. Every library
// call consumes the status of its own HIP calls, so an error still pending
// right before a launch was left by someone else: take_stray_error records
// it (with `where`) and clears it, so that the launch reports only its own
// status. (Device faults are sticky and are still reported by the launch.)
void take_stray_error(const char *where);

// ---- kernel launchers (kernels.hip) ---------------------------------------
hipError_t launch_init(uint64_t *state, uint32_t n, const SeedMix &mix, hipStream_t s);
hipError_t launch_gen(const rngx_launch &cfg, bool u32, bool star, uint64_t *state, uint32_t n,
                      uint32_t iters, void *out, hipStream_t s);
bool launch_cfg_valid(const rngx_launch &cfg);
// copy.hip: device buffer -> page-locked host memory (device-mapped address).
hipError_t launch_d2h(const void *src, void *dst_mapped, size_t bytes, uint32_t blocks,
                      hipStream_t s);

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
    rngx_launch cfg64{512, 2, 1, 7000}; // row-scheduled; see rngx_launch in rngx.h
    rngx_launch cfg32{0, 0, 0, 0};      // block 0: the library's choice (generate_locked)
    // Streams and events of the device-to-host pipeline (pipeline.cpp).
    hipStream_t pipe_gen = nullptr, pipe_copy = nullptr;
    hipEvent_t copy_done[2] = {nullptr, nullptr};
    int copy_mode = RNGX_COPY_KERNEL;
    // 16 workgroups saturate PCIe 5.0 x16 on MI355X and slow the overlapping
    // generation kernel least (measured: 16 to 256 all within 4 %).
    uint32_t copy_blocks = 16;
    // rngx_inject_copy_failure: step of the next streamed run whose copy
    // fails (UINT64_MAX: none).
    uint64_t fail_copy_at = UINT64_MAX;
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
// The same, returning the end event it recorded (nullptr if none): a caller
// may order other streams after the operation with it instead of recording
// an event of its own. The event stays valid until the profiling window is
// restarted, which needs the generator lock.
hipEvent_t end_event(int token, hipStream_t s);
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
// Write an event table as text or Chrome trace JSON (RNGX_EXPORT_*).
int write_table(const rngx_prof_event *events, uint32_t n, const char *path, int format);

} // namespace rngx
