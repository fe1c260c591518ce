// Host side of the batched path: request packing, work-item numbering,
// HIP-graph capture and replay, the autotuner, and the device checksum.
//
// A BatchSlot owns one page-locked staging buffer and one device table
// (a BatchDesc followed by the packed BatchReq array). A batch is staged on
// the host, then one HIP graph copies the table to the device and launches
// the persistent kernel; the graph is captured once per (capacity, launch
// configuration) and replayed for every later batch, because the kernel
// reads everything that changes from the device table. Before a slot's
// staging buffer is rewritten, the slot's previous batch must have finished
// (its `done` event).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.h"

namespace rngx {

namespace {

const uint32_t kValuesPerLane[8] = {8, 16, 32, 64, 128, 256, 512, 1024};
constexpr int kNumS = 8;
// Wavefronts per group of the grouped order (rngx_batch_cfg.group).
const uint32_t kGroupSizes[4] = {16, 32, 64, 128};
constexpr int kNumGroups = 4;

} // namespace

int batch_s_index(uint32_t s)
{
    for (int i = 0; i < kNumS; ++i)
        if (kValuesPerLane[i] == s)
            return i;
    return -1;
}

int batch_group_index(uint32_t g)
{
    for (int i = 0; i < kNumGroups; ++i)
        if (kGroupSizes[i] == g)
            return i;
    return -1;
}

// The constant tables every batch launch reads, in static device memory: one
// copy per device, which lives as long as the process (1,136 KiB). They are
// filled on a device's first batched call of any kind, so later calls, also
// the allocation-free entry point, only enqueue work.
__device__ __align__(256) uint64_t g_pow2[64 * 64];                  // T^(2^b), 64 rows each
__device__ __align__(256) uint64_t g_spread[kNumS * kSpreadTable];   // lane-spread tables per S
__device__ __align__(256) uint64_t g_carry_nib[kNumS * kCarryTable]; // T^(63 S) nibble tables per S
// T^(g 64 S - S) nibble tables per S and group size g (the grouped order).
__device__ __align__(256) uint64_t g_group_nib[kNumS * kNumGroups * kCarryTable];

namespace {

// Per-device bookkeeping: the device addresses of the static tables once
// they are filled there, and the checksum accumulator (allocated on the
// first checksum, freed by rngx_shutdown).
struct DevTables {
    int n_cus = 0;
    bool loaded = false;
    const uint64_t *d_pow2 = nullptr;
    const uint64_t *d_spread = nullptr;
    const uint64_t *d_carry_nib = nullptr;
    const uint64_t *d_group_nib = nullptr;
    int clock_khz = 0;               // constant-rate clock (s_memrealtime)
    uint64_t *d_acc = nullptr;       // checksum accumulator
    uint64_t *h_acc = nullptr;       // page-locked copy of it
};
constexpr int kMaxDevices = 64;

struct BatchGlobals {
    std::mutex mu;
    DevTables dev[kMaxDevices];
    // The grouped order: the autotuner's pick on the 4,096-stream table and
    // the server's order for large batches (6.2 TB/s there against 5.9 for
    // the persistent grid with S = 256).
    rngx_batch_cfg cfg{16, 4, 0, 1, 16, 0, 0, 32, 8, 6250};
    BatchSlot api_slot;
    // Device address of `scratch` per device (rngx_generate_batch_noalloc),
    // taken once on the device's first such call.
    unsigned char *scratch_ptr[kMaxDevices] = {};
};

// Request table of rngx_generate_batch_noalloc: a BatchDesc, then up to
// RNGX_NOALLOC_MAX_REQS records at kReqOffset (262,272 bytes). One copy per
// device, held until the process ends; every such call on a device rewrites
// it, so calls that overlap on one device race. In host code the name is a
// stand-in for the symbol, never a device address: the address comes from
// hipGetSymbolAddress (scratch_ptr above).
constexpr size_t kScratchBytes = kReqOffset + (size_t)RNGX_NOALLOC_MAX_REQS * sizeof(BatchReq);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
// Its host image, built under the batch lock and copied with one
// hipMemcpyAsync. The copy is from pageable memory, which HIP performs
// synchronously, so the image may be rewritten as soon as the copy returns.
alignas(256) unsigned char g_noalloc_host[kScratchBytes];

BatchGlobals &G()
{
    static BatchGlobals *g = new BatchGlobals;
    return *g;
}

// Free the checksum accumulator (the static tables stay filled).
void free_acc(DevTables &t)
{
    if (t.d_acc)
        RNGX_NOTE(hipFree(t.d_acc));
    if (t.h_acc)
        RNGX_NOTE(hipHostFree(t.h_acc));
    t.d_acc = nullptr;
    t.h_acc = nullptr;
}

// Host images of the lane-spread and carry tables for every allowed S, in
// static host memory (built under tables_mu, once per device): filling the
// device tables allocates nothing.
uint64_t g_spread_host[kNumS * kSpreadTable];
uint64_t g_carry_host[kNumS * kCarryTable];
uint64_t g_group_host[kNumS * kNumGroups * kCarryTable];

// M = T^k as 16 tables of 16 entries: entry v of table q is M (v << 4q), so
// M x is the XOR of 16 lookups, one per nibble of x.
void nibble_table(uint64_t k, uint64_t *t)
{
    uint64_t rows[64], col[64] = {0};
    power_rows(k, rows);
    for (int r = 0; r < 64; ++r)
        for (int j = 0; j < 64; ++j)
            col[j] |= ((rows[r] >> j) & 1u) << r;
    for (int q = 0; q < 16; ++q)
        for (int v = 0; v < 16; ++v) {
            uint64_t e = 0;
            for (int b = 0; b < 4; ++b)
                if ((v >> b) & 1)
                    e ^= col[4 * q + b];
            t[16 * q + v] = e;
        }
}

void build_host_tables(uint64_t *spread, uint64_t *nib, uint64_t *group)
{
    std::memset(spread, 0, sizeof(uint64_t) * kNumS * kSpreadTable);
    std::memset(nib, 0, sizeof(uint64_t) * kNumS * kCarryTable);
    // Grouped order: a lane that just emitted its S values of a tile moves
    // to the tile g tiles on, g C - S values further.
    for (int i = 0; i < kNumS; ++i)
        for (int gi = 0; gi < kNumGroups; ++gi)
            nibble_table((uint64_t)kGroupSizes[gi] * 64 * kValuesPerLane[i] - kValuesPerLane[i],
                         group + ((size_t)i * kNumGroups + gi) * kCarryTable);
    for (int i = 0; i < kNumS; ++i) {
        const uint64_t S = kValuesPerLane[i];
        // Lane spread: entry ((16 q + v) * 64 + m) is T^(m S) (v << 4q),
        // so a lane m places above a wave-uniform state z with the XOR of
        // one entry per nibble of z.
        uint64_t *sp = spread + (size_t)kSpreadTable * i;
        for (uint32_t m = 0; m < 64; ++m) {
            uint64_t rows[64], col[64] = {0};
            power_rows(m * S, rows);
            for (int r = 0; r < 64; ++r)
                for (int j = 0; j < 64; ++j)
                    col[j] |= ((rows[r] >> j) & 1u) << r;
            for (int q = 0; q < 16; ++q)
                for (int v = 0; v < 16; ++v) {
                    uint64_t e = 0;
                    for (int b = 0; b < 4; ++b)
                        if ((v >> b) & 1)
                            e ^= col[4 * q + b];
                    sp[(16 * q + v) * 64 + m] = e;
                }
        }
        // A lane that just emitted its S values of a tile is C - S = 63 S
        // values short of its start in the next tile. M = T^(63 S) is
        // stored as 16 tables of 16 entries: entry v of table q is
        // M (v << 4q), so M x is the XOR of 16 lookups, one per nibble.
        uint64_t carry_rows[64];
        power_rows(63ull * S, carry_rows);
        uint64_t col[64] = {0};
        for (int r = 0; r < 64; ++r)
            for (int j = 0; j < 64; ++j)
                col[j] |= ((carry_rows[r] >> j) & 1u) << r;
        uint64_t *t = nib + (size_t)kCarryTable * i;
        for (int q = 0; q < 16; ++q)
            for (int v = 0; v < 16; ++v)
                for (int b = 0; b < 4; ++b)
                    if ((v >> b) & 1)
                        t[16 * q + v] ^= col[4 * q + b];
    }
}

void free_slot(BatchSlot &s)
{
    if (s.done)
        RNGX_NOTE(hipEventSynchronize(s.done));
    if (s.exec)
        RNGX_NOTE(hipGraphExecDestroy(s.exec));
    if (s.staging)
        RNGX_NOTE(hipHostFree(s.staging));
    if (s.devtab)
        RNGX_NOTE(hipFree(s.devtab));
    if (s.done)
        RNGX_NOTE(hipEventDestroy(s.done));
    if (s.cap_stream)
        RNGX_NOTE(hipStreamDestroy(s.cap_stream));
    s = BatchSlot();
}

std::mutex &tables_mu()
{
    static std::mutex *m = new std::mutex;
    return *m;
}

} // namespace

int batch_tables_locked(const uint64_t **pow2, const uint64_t **spread_all, int *n_cus,
                        const uint64_t **carry_nib_all, const uint64_t **group_nib_all,
                        int *clock_khz)
{
    // Own lock: the server thread reaches here without the batch API lock.
    std::lock_guard<std::mutex> lk(tables_mu());
    BatchGlobals &g = G();
    int dev = -1;
    RNGX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(RNGX_E_INVAL, "batch: device %d is beyond the %d the library supports",
                         dev, kMaxDevices);
    DevTables &t = g.dev[dev];
    if (!t.loaded) {
        // Device addresses of this device's copies of the static tables
        // (the arrays' names are host-side stand-ins), then their contents.
        build_host_tables(g_spread_host, g_carry_host, g_group_host);
        void *p2 = nullptr, *ps = nullptr, *pc = nullptr, *pg = nullptr;
        int cus = 0, khz = 0;
        hipError_t e = hipGetSymbolAddress(&p2, HIP_SYMBOL(g_pow2));
        if (e == hipSuccess)
            e = hipGetSymbolAddress(&ps, HIP_SYMBOL(g_spread));
        if (e == hipSuccess)
            e = hipGetSymbolAddress(&pc, HIP_SYMBOL(g_carry_nib));
        if (e == hipSuccess)
            e = hipGetSymbolAddress(&pg, HIP_SYMBOL(g_group_nib));
        if (e == hipSuccess)
            e = hipMemcpy(p2, jump_tables(), sizeof g_pow2, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(ps, g_spread_host, sizeof g_spread, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pc, g_carry_host, sizeof g_carry_nib, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pg, g_group_host, sizeof g_group_nib, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
        if (e != hipSuccess)
            return hip_fail(e, "batch: device tables");
        t.d_pow2 = static_cast<const uint64_t *>(p2);
        t.d_spread = static_cast<const uint64_t *>(ps);
        t.d_carry_nib = static_cast<const uint64_t *>(pc);
        t.d_group_nib = static_cast<const uint64_t *>(pg);
        t.clock_khz = khz > 0 ? khz : 100000;
        t.n_cus = cus;
        t.loaded = true;
    }
    if (pow2)
        *pow2 = t.d_pow2;
    if (spread_all)
        *spread_all = t.d_spread;
    if (carry_nib_all)
        *carry_nib_all = t.d_carry_nib;
    if (group_nib_all)
        *group_nib_all = t.d_group_nib;
    if (clock_khz)
        *clock_khz = t.clock_khz;
    if (n_cus)
        *n_cus = t.n_cus;
    return RNGX_OK;
}

int resolve_batch_cfg(const rngx_batch_cfg &c, int n_cus, rngx_batch_cfg *out)
{
    rngx_batch_cfg r = c;
    if (r.group) {
        // Every block that fits at once, rounded down to whole groups.
        int occ = 0;
        const hipError_t e = batch_group_occupancy(r, &occ);
        if (e != hipSuccess)
            return hip_fail(e, "batch: occupancy of the grouped kernel");
        const uint64_t per_group = r.group / r.waves_per_block;
        const uint64_t fit = (uint64_t)std::max(1, occ) * (uint64_t)std::max(1, n_cus);
        r.blocks = (uint32_t)std::max<uint64_t>(per_group, fit / per_group * per_group);
    } else if (r.blocks == 0) { // 8 waves per compute unit: the autotuner's usual pick
        r.blocks = (uint32_t)std::max(1, n_cus * 8 / (int)r.waves_per_block);
    }
    *out = r;
    return RNGX_OK;
}

void fill_batch_tables(BatchTables &t, const rngx_batch_cfg &cfg, const uint64_t *pow2,
                       const uint64_t *spread_all, const uint64_t *nib_all,
                       const uint64_t *group_all, int clock_khz)
{
    const int si = batch_s_index(cfg.values_per_lane);
    t.pow2 = pow2;
    t.spread = spread_all + (size_t)kSpreadTable * si;
    t.carry_nib = nib_all + (size_t)kCarryTable * si;
    t.group_nib = cfg.group ? group_all + ((size_t)si * kNumGroups +
                                           batch_group_index(cfg.group)) * kCarryTable
                            : nullptr;
    t.clock_khz = (uint32_t)clock_khz;
}

int batch_stage_items(BatchSlot &slot, const StageReq *items, uint32_t k,
                      uint32_t values_per_lane, const uint64_t *states)
{
    // A slot's buffers, event and graph belong to the device they were made
    // on; when another device is current, the slot starts over there.
    int dev = -1;
    RNGX_HIP(hipGetDevice(&dev));
    if (slot.device != dev) {
        free_slot(slot);
        slot.device = dev;
    }
    // Grow the slot to a power-of-two capacity (>= 64 requests).
    if (k > slot.capacity || !slot.staging) {
        uint32_t cap = 64;
        while (cap < k)
            cap <<= 1;
        if (slot.done)
            RNGX_HIP(hipEventSynchronize(slot.done));
        if (slot.exec) {
            RNGX_NOTE(hipGraphExecDestroy(slot.exec));
            slot.exec = nullptr;
        }
        if (slot.staging)
            RNGX_NOTE(hipHostFree(slot.staging));
        if (slot.devtab)
            RNGX_NOTE(hipFree(slot.devtab));
        slot.staging = slot.devtab = nullptr;
        slot.capacity = 0;
        const size_t bytes = kReqOffset + (size_t)cap * sizeof(BatchReq);
        hipError_t e = hipHostMalloc(&slot.staging, bytes, hipHostMallocDefault);
        if (e != hipSuccess) {
            slot.staging = nullptr;
            return hip_fail(e, "hipHostMalloc (batch staging)");
        }
        e = hipMalloc(&slot.devtab, bytes);
        if (e != hipSuccess) {
            RNGX_NOTE(hipHostFree(slot.staging));
            slot.staging = slot.devtab = nullptr;
            return hip_fail(e, "hipMalloc (batch table)");
        }
        slot.capacity = cap;
    }
    if (!slot.done)
        RNGX_HIP(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    // The slot's previous batch must have read its table before we rewrite it.
    RNGX_HIP(hipEventSynchronize(slot.done));

    const uint64_t C = 64ull * values_per_lane;
    BatchDesc *desc = static_cast<BatchDesc *>(slot.staging);
    BatchReq *tab = reinterpret_cast<BatchReq *>(static_cast<char *>(slot.staging) + kReqOffset);
    uint64_t n_items = 0;
    for (uint32_t j = 0; j < k; ++j) {
        const StageReq &q = items[j];
        n_items += make_record(tab[j], q.offset, q.length, q.vbase, n_items, q.gid, q.mix, q.dst,
                               C);
    }
    std::memset(desc, 0, sizeof *desc);
    desc->reqs = reinterpret_cast<const BatchReq *>(static_cast<char *>(slot.devtab) +
                                                    kReqOffset);
    desc->states = states;
    desc->n_items = n_items;
    desc->m = k;
    slot.m_staged = k;
    slot.n_items = n_items;
    return RNGX_OK;
}

int batch_validate(const rngx_req *reqs, uint32_t m, const uint64_t *out, uint64_t out_cap,
                   uint64_t *total_out)
{
    if (m && !reqs)
        return set_error(RNGX_E_INVAL, "batch: reqs is NULL");
    unsigned __int128 total = 0;
    for (uint32_t j = 0; j < m; ++j) {
        if (reqs[j].reserved)
            return set_error(RNGX_E_INVAL, "batch: request %u has a nonzero reserved field", j);
        if (reqs[j].length && reqs[j].offset > UINT64_MAX - (reqs[j].length - 1))
            return set_error(RNGX_E_INVAL,
                             "batch: request %u runs past value number 2^64 - 1", j);
        total += reqs[j].length;
    }
    if (total > (unsigned __int128)UINT64_MAX / 8)
        return set_error(RNGX_E_INVAL, "batch: total length overflows");
    if ((uint64_t)total > out_cap)
        return set_error(RNGX_E_INVAL, "batch: requests need %llu values but out holds %llu",
                         (unsigned long long)total, (unsigned long long)out_cap);
    if (total && !out)
        return set_error(RNGX_E_INVAL, "batch: out is NULL");
    if (total && (reinterpret_cast<uintptr_t>(out) & 15u))
        return set_error(RNGX_E_INVAL, "batch: out is not 16-byte aligned");
    *total_out = (uint64_t)total;
    return RNGX_OK;
}

// Values between the start of out's 128-byte line and out (even: out is
// 16-byte aligned). A packed batch's virtual index space starts there: the
// kernel writes each row of 16 values to the 128 bytes at virtual indices
// 16 j .. 16 j + 15, which are then one whole cache line of the output. With
// the virtual index equal to the output index, every row of an output that
// is 16- but not 128-byte aligned would straddle two lines, which measured
// 1.4 times the algorithmic bytes in DRAM writes and half the write rate.
static uint64_t line_skew(const uint64_t *out)
{
    return (reinterpret_cast<uintptr_t>(out) & 127u) / sizeof(uint64_t);
}

int batch_stage(BatchSlot &slot, const rngx_req *reqs, uint32_t m, uint64_t *out,
                uint64_t out_cap, uint32_t values_per_lane, uint64_t *total_out)
{
    int rc = batch_validate(reqs, m, out, out_cap, total_out);
    if (rc || *total_out == 0)
        return rc;
    // Packed layout: the virtual index of a value is its output index plus
    // the skew of `out` in its 128-byte line, so tile rows fall on whole
    // lines of the output.
    std::vector<StageReq> items;
    items.reserve(m);
    const uint64_t skew = line_skew(out);
    uint64_t base = 0;
    for (uint32_t j = 0; j < m; ++j) {
        const uint64_t len = reqs[j].length;
        if (len) {
            StageReq q;
            q.offset = reqs[j].offset;
            q.length = len;
            q.vbase = skew + base;
            q.dst = out + base;
            q.gid = reqs[j].gid;
            q.mix = seed_mix(reqs[j].seed);
            items.push_back(q);
        }
        base += len;
    }
    return batch_stage_items(slot, items.data(), (uint32_t)items.size(), values_per_lane,
                             nullptr);
}

int batch_launch(BatchSlot &slot, const rngx_batch_cfg &cfg_in, bool star, hipStream_t stream,
                 bool fit_grid, const char *prof_name)
{
    const uint64_t *pow2 = nullptr, *spread_all = nullptr, *nib_all = nullptr, *group_all = nullptr;
    int n_cus = 0, clock_khz = 0;
    int rc = batch_tables_locked(&pow2, &spread_all, &n_cus, &nib_all, &group_all, &clock_khz);
    if (rc)
        return rc;
    rngx_batch_cfg cfg;
    if ((rc = resolve_batch_cfg(cfg_in, n_cus, &cfg)))
        return rc;
    if (cfg.per_item) {
        // One wave per item: the grid follows the item count (a captured
        // graph is re-captured when that count changes).
        const uint64_t need = (slot.n_items + cfg.waves_per_block - 1) / cfg.waves_per_block;
        if (need > 0x7fffffffull)
            return set_error(RNGX_E_INVAL, "batch: %llu work items exceed one grid",
                             (unsigned long long)slot.n_items);
        cfg.blocks = (uint32_t)std::max<uint64_t>(1, need);
    } else if (fit_grid && !cfg.use_graph && !cfg.group) {
        const uint64_t need = (slot.n_items + cfg.waves_per_block - 1) / cfg.waves_per_block;
        if (need < cfg.blocks)
            cfg.blocks = (uint32_t)std::max<uint64_t>(1, need);
    }
    BatchTables tabs;
    fill_batch_tables(tabs, cfg, pow2, spread_all, nib_all, group_all, clock_khz);
    const BatchDesc *ddesc = static_cast<const BatchDesc *>(slot.devtab);
    const int tok = prof::begin(prof_name, stream);
    if (cfg.use_graph) {
        const bool same = slot.exec && slot.exec_cfg.values_per_lane == cfg.values_per_lane &&
                          slot.exec_cfg.waves_per_block == cfg.waves_per_block &&
                          slot.exec_cfg.blocks == cfg.blocks &&
                          slot.exec_cfg.row_values == cfg.row_values &&
                          slot.exec_cfg.run_items == cfg.run_items &&
                          slot.exec_cfg.per_item == cfg.per_item &&
                          slot.exec_cfg.group == cfg.group &&
                          slot.exec_cfg.group_steps == cfg.group_steps &&
                          slot.exec_cfg.pace_gbs == cfg.pace_gbs && slot.exec_star == star;
        if (!same) {
            if (slot.exec) {
                RNGX_NOTE(hipGraphExecDestroy(slot.exec));
                slot.exec = nullptr;
            }
            if (!slot.cap_stream)
                RNGX_HIP(hipStreamCreateWithFlags(&slot.cap_stream, hipStreamNonBlocking));
            const size_t bytes = kReqOffset + (size_t)slot.capacity * sizeof(BatchReq);
            // Relaxed mode: a capture the library opens must never make a
            // HIP call of another thread (a server's scheduler, the
            // application's allocator) fail as unsafe during capture. The
            // window holds only the table copy and the launch, which every
            // mode allows.
            RNGX_HIP(hipStreamBeginCapture(slot.cap_stream, hipStreamCaptureModeRelaxed));
            hipError_t e1 = hipMemcpyAsync(slot.devtab, slot.staging, bytes,
                                           hipMemcpyHostToDevice, slot.cap_stream);
            // (e1 is consumed here if it failed: it is reported below.)
            take_stray_error("before the captured batch kernel launch");
            hipError_t e2 = launch_batch(cfg, ddesc, tabs, star, slot.cap_stream);
            hipGraph_t graph = nullptr;
            hipError_t e3 = hipStreamEndCapture(slot.cap_stream, &graph);
            if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
                if (graph)
                    RNGX_NOTE(hipGraphDestroy(graph));
                return hip_fail(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3),
                                "batch graph capture");
            }
            hipError_t e4 = hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0);
            RNGX_NOTE(hipGraphDestroy(graph));
            if (e4 != hipSuccess) {
                slot.exec = nullptr;
                return hip_fail(e4, "hipGraphInstantiate (batch)");
            }
            slot.exec_cfg = cfg;
            slot.exec_star = star;
        }
        RNGX_HIP(hipGraphLaunch(slot.exec, stream));
    } else if (cfg.per_item && slot.m_staged <= kSmallReqs) {
        // Small table: it goes in the kernel's arguments, no upload.
        SmallTable st;
        std::memcpy(&st.desc, slot.staging, sizeof(BatchDesc));
        std::memcpy(st.reqs, static_cast<const char *>(slot.staging) + kReqOffset,
                    (size_t)slot.m_staged * sizeof(BatchReq));
        take_stray_error("before the batch kernel launch");
        hipError_t e = launch_batch_small(cfg, st, tabs, star, stream);
        if (e != hipSuccess)
            return hip_fail(e, "batch kernel launch");
    } else {
        const size_t bytes = kReqOffset + (size_t)slot.m_staged * sizeof(BatchReq);
        RNGX_HIP(hipMemcpyAsync(slot.devtab, slot.staging, bytes, hipMemcpyHostToDevice, stream));
        take_stray_error("before the batch kernel launch");
        hipError_t e = launch_batch(cfg, ddesc, tabs, star, stream);
        if (e != hipSuccess)
            return hip_fail(e, "batch kernel launch");
    }
    prof::end(tok, stream);
    RNGX_HIP(hipEventRecord(slot.done, stream));
    return RNGX_OK;
}

void release_slot(BatchSlot &slot) { free_slot(slot); }

void release_batch()
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    free_slot(g.api_slot);
    std::lock_guard<std::mutex> lt(tables_mu());
    int cur = -1;
    RNGX_NOTE(hipGetDevice(&cur));
    for (int d = 0; d < kMaxDevices; ++d) {
        if (!g.dev[d].d_acc && !g.dev[d].h_acc)
            continue;
        RNGX_NOTE(hipSetDevice(d));
        free_acc(g.dev[d]);
    }
    if (cur >= 0)
        RNGX_NOTE(hipSetDevice(cur));
}

// Device address of this device's `scratch` (once per device, under the
// batch lock).
int noalloc_scratch_locked(BatchGlobals &g, int dev, unsigned char **ptr)
{
    if (!g.scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress (batch scratch)");
        g.scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *ptr = g.scratch_ptr[dev];
    return RNGX_OK;
}

rngx_batch_cfg current_batch_cfg()
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    return g.cfg;
}

int checksum_locked(const uint64_t *data, uint64_t n, hipStream_t s, uint64_t *result)
{
    int rc = batch_tables_locked(nullptr, nullptr, nullptr);
    if (rc)
        return rc;
    int dev = -1;
    RNGX_HIP(hipGetDevice(&dev));
    DevTables &t = G().dev[dev];
    {
        std::lock_guard<std::mutex> lt(tables_mu());
        if (!t.d_acc) {
            void *d = nullptr, *h = nullptr;
            hipError_t e = hipMalloc(&d, sizeof(uint64_t));
            if (e != hipSuccess)
                return hip_fail(e, "checksum: hipMalloc (accumulator)");
            e = hipHostMalloc(&h, sizeof(uint64_t), hipHostMallocDefault);
            if (e != hipSuccess) {
                RNGX_NOTE(hipFree(d));
                return hip_fail(e, "checksum: hipHostMalloc (accumulator)");
            }
            t.d_acc = static_cast<uint64_t *>(d);
            t.h_acc = static_cast<uint64_t *>(h);
        }
    }
    RNGX_HIP(hipMemsetAsync(t.d_acc, 0, sizeof(uint64_t), s));
    take_stray_error("before the checksum kernel launch");
    RNGX_HIP(launch_checksum(data, n, t.d_acc, s));
    RNGX_HIP(hipMemcpyAsync(t.h_acc, t.d_acc, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    RNGX_HIP(hipStreamSynchronize(s));
    *result = *t.h_acc;
    return RNGX_OK;
}

} // namespace rngx

using namespace rngx;

extern "C" int rngx_generate_batch(const rngx_req *reqs, uint32_t m, uint64_t *out,
                                   uint64_t out_cap, void *stream)
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    clear_error();
    uint64_t total = 0;
    int rc = batch_stage(g.api_slot, reqs, m, out, out_cap, g.cfg.values_per_lane, &total);
    if (rc)
        return rc;
    if (total == 0)
        return RNGX_OK;
    return batch_launch(g.api_slot, g.cfg, current_scrambler() == RNGX_SCRAMBLE_STAR,
                        static_cast<hipStream_t>(stream));
}

extern "C" int rngx_generate_batch_noalloc(const rngx_req *reqs, uint32_t m, uint64_t *out,
                                           uint64_t out_cap, void *stream)
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    clear_error();
    if (m > RNGX_NOALLOC_MAX_REQS)
        return set_error(RNGX_E_INVAL,
                         "rngx_generate_batch_noalloc: %u requests exceed the limit of %u", m,
                         (unsigned)RNGX_NOALLOC_MAX_REQS);
    uint64_t total = 0;
    int rc = batch_validate(reqs, m, out, out_cap, &total);
    if (rc || total == 0)
        return rc;
    int dev = -1;
    RNGX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(RNGX_E_INVAL, "batch: device %d is beyond the %d the library supports",
                         dev, kMaxDevices);
    unsigned char *dscratch = nullptr;
    rc = noalloc_scratch_locked(g, dev, &dscratch);
    if (rc)
        return rc;
    // The jump tables are static device arrays too; the device's first
    // batched call of any kind fills them.
    const uint64_t *pow2 = nullptr, *spread_all = nullptr, *nib_all = nullptr, *group_all = nullptr;
    int n_cus = 0, clock_khz = 0;
    rc = batch_tables_locked(&pow2, &spread_all, &n_cus, &nib_all, &group_all, &clock_khz);
    if (rc)
        return rc;
    rngx_batch_cfg cfg;
    if ((rc = resolve_batch_cfg(g.cfg, n_cus, &cfg)))
        return rc;
    const uint64_t C = 64ull * cfg.values_per_lane;

    // The table, staged as the allocating call stages it (packed layout
    // with the output's line skew; empty requests dropped).
    BatchDesc *desc = reinterpret_cast<BatchDesc *>(g_noalloc_host);
    BatchReq *tab = reinterpret_cast<BatchReq *>(g_noalloc_host + kReqOffset);
    const uint64_t skew = line_skew(out);
    uint32_t k = 0;
    uint64_t base = 0, n_items = 0;
    for (uint32_t j = 0; j < m; ++j) {
        const uint64_t len = reqs[j].length;
        if (len) {
            n_items += make_record(tab[k], reqs[j].offset, len, skew + base, n_items, reqs[j].gid,
                                   seed_mix(reqs[j].seed), out + base, C);
            ++k;
        }
        base += len;
    }
    std::memset(desc, 0, sizeof *desc); // next_item = 0: the upload resets the work counter
    desc->reqs = reinterpret_cast<const BatchReq *>(dscratch + kReqOffset);
    desc->states = nullptr;
    desc->n_items = n_items;
    desc->m = k;

    const uint64_t need = (n_items + cfg.waves_per_block - 1) / cfg.waves_per_block;
    if (cfg.per_item) {
        if (need > 0x7fffffffull)
            return set_error(RNGX_E_INVAL, "batch: %llu work items exceed one grid",
                             (unsigned long long)n_items);
        cfg.blocks = (uint32_t)std::max<uint64_t>(1, need);
    } else if (need < cfg.blocks && !cfg.group) {
        cfg.blocks = (uint32_t)std::max<uint64_t>(1, need);
    }
    BatchTables tabs;
    fill_batch_tables(tabs, cfg, pow2, spread_all, nib_all, group_all, clock_khz);
    const bool star = current_scrambler() == RNGX_SCRAMBLE_STAR;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (cfg.per_item && k <= kSmallReqs) {
        SmallTable st;
        std::memcpy(&st.desc, desc, sizeof(BatchDesc));
        std::memcpy(st.reqs, tab, (size_t)k * sizeof(BatchReq));
        take_stray_error("before the allocation-free batch kernel launch");
        hipError_t e = launch_batch_small(cfg, st, tabs, star, s);
        if (e != hipSuccess)
            return hip_fail(e, "batch kernel launch");
        return RNGX_OK;
    }
    RNGX_HIP(hipMemcpyAsync(dscratch, g_noalloc_host, kReqOffset + (size_t)k * sizeof(BatchReq),
                            hipMemcpyHostToDevice, s));
    take_stray_error("before the allocation-free batch kernel launch");
    hipError_t e = launch_batch(cfg, reinterpret_cast<const BatchDesc *>(dscratch), tabs, star, s);
    if (e != hipSuccess)
        return hip_fail(e, "batch kernel launch");
    return RNGX_OK;
}

extern "C" int rngx_set_batch_cfg(const rngx_batch_cfg *cfg)
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    clear_error();
    if (!cfg || !batch_cfg_valid(*cfg))
        return set_error(RNGX_E_INVAL,
                         "rngx_set_batch_cfg: values_per_lane must be 8, 16, 32, 64, 128, 256, "
                         "512 or 1024, waves_per_block 1..4, blocks 0..65536 (0 = 8 waves per "
                         "compute unit), use_graph 0/1, row_values 8 or 16 (at most "
                         "values_per_lane), run_items 0..64, per_item 0/1; group 0, 16, 32, 64 "
                         "or 128 (a multiple of waves_per_block, per_item 0) with group_steps "
                         "1..256 and pace_gbs 0 or 1000..20000, else group_steps and pace_gbs 0");
    g.cfg = *cfg;
    return RNGX_OK;
}

extern "C" int rngx_get_batch_cfg(rngx_batch_cfg *cfg)
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    clear_error();
    if (!cfg)
        return set_error(RNGX_E_INVAL, "rngx_get_batch_cfg: NULL");
    *cfg = g.cfg;
    return RNGX_OK;
}

extern "C" int rngx_checksum(const uint64_t *data, uint64_t n, void *stream, uint64_t *result)
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    clear_error();
    if (!result)
        return set_error(RNGX_E_INVAL, "rngx_checksum: result is NULL");
    if (n && !data)
        return set_error(RNGX_E_INVAL, "rngx_checksum: data is NULL");
    return checksum_locked(data, n, static_cast<hipStream_t>(stream), result);
}

extern "C" int rngx_autotune_batch(const rngx_req *reqs, uint32_t m, uint64_t *out,
                                   uint64_t out_cap, uint32_t reps, void *stream,
                                   rngx_tune_result *result)
{
    BatchGlobals &g = G();
    std::lock_guard<std::mutex> lk(g.mu);
    clear_error();
    if (!result)
        return set_error(RNGX_E_INVAL, "rngx_autotune_batch: result is NULL");
    if (reps == 0)
        return set_error(RNGX_E_INVAL, "rngx_autotune_batch: reps must be >= 1");
    int n_cus = 0;
    int rc = batch_tables_locked(nullptr, nullptr, &n_cus);
    if (rc)
        return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool star = current_scrambler() == RNGX_SCRAMBLE_STAR;
    std::memset(result, 0, sizeof *result);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RNGX_HIP(hipEventCreate(&e0));
    RNGX_HIP(hipEventCreate(&e1));
    struct Events {
        hipEvent_t a, b;
        ~Events()
        {
            RNGX_NOTE(hipEventDestroy(a));
            RNGX_NOTE(hipEventDestroy(b));
        }
    } guard{e0, e1};

    uint64_t ref_sum = 0, total = 0;
    bool have_ref = false;
    double best = 1e300;
    // The persistent launch (one grid that takes work items from a counter):
    // values_per_lane x run length x waves_per_block x waves per compute
    // unit, all with 128-byte rows (64-byte rows write half cache lines and
    // were much slower in every measurement); combinations whose LDS would
    // not fit the waves per CU are skipped. One wave per item is not a
    // candidate: it is a configuration of its own (rngx_set_batch_cfg) and
    // the server's schedule for small batches.
    auto try_cfg = [&](const rngx_batch_cfg &c) -> int {
        int rc2 = batch_stage(g.api_slot, reqs, m, out, out_cap, c.values_per_lane, &total);
        if (rc2)
            return rc2;
        if (total == 0)
            return set_error(RNGX_E_INVAL, "rngx_autotune_batch: no values requested");
        rc2 = batch_launch(g.api_slot, c, star, s); // warm-up (and graph capture)
        if (rc2)
            return rc2;
        uint64_t sum = 0;
        rc2 = checksum_locked(out, total, s, &sum);
        if (rc2)
            return rc2;
        if (!have_ref) {
            ref_sum = sum;
            have_ref = true;
        } else if (sum != ref_sum) {
            return set_error(RNGX_E_HIP,
                             "autotune: configuration (S=%u, waves/block=%u, blocks=%u, "
                             "group=%u, steps=%u, pace=%u) produced a different output",
                             c.values_per_lane, c.waves_per_block, c.blocks, c.group,
                             c.group_steps, c.pace_gbs);
        }
        RNGX_HIP(hipEventRecord(e0, s));
        for (uint32_t r = 0; r < reps; ++r) {
            rc2 = batch_launch(g.api_slot, c, star, s);
            if (rc2)
                return rc2;
        }
        RNGX_HIP(hipEventRecord(e1, s));
        RNGX_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RNGX_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double mean = (double)ms / reps;
        if (result->n_tried < RNGX_TUNE_MAX) {
            result->tried[result->n_tried].cfg = c;
            result->tried[result->n_tried].ms = mean;
        }
        ++result->n_tried;
        if (mean < best) {
            best = mean;
            result->best = c;
        }
        return RNGX_OK;
    };
    const uint32_t svals[4] = {64, 128, 256, 512};
    const uint32_t runs[2] = {1, 8};
    const uint32_t wpbs[2] = {2, 4};
    const uint32_t waves_per_cu[3] = {8, 16, 32};
    const uint32_t row = 16;
    for (uint32_t si = 0; si < 4; ++si) {
        for (uint32_t ui = 0; ui < 2; ++ui) {
            for (uint32_t wi = 0; wi < 2; ++wi) {
                for (uint32_t oi = 0; oi < 3; ++oi) {
                    const uint32_t lds_per_block = 8u * (kCarryTable + wpbs[wi] * 64u * (row + 2));
                    if (waves_per_cu[oi] / wpbs[wi] * lds_per_block > 160u * 1024u)
                        continue;
                    rngx_batch_cfg c{};
                    c.values_per_lane = svals[si];
                    c.waves_per_block = wpbs[wi];
                    c.blocks = (uint32_t)std::max(1, n_cus * (int)waves_per_cu[oi] / (int)wpbs[wi]);
                    c.use_graph = g.cfg.use_graph;
                    c.row_values = row;
                    c.run_items = runs[ui];
                    c.per_item = 0;
                    if ((rc = try_cfg(c)))
                        return rc;
                }
            }
        }
    }
    // The grouped order with S = 16 (128-byte rows, 4 waves per block):
    // groups of 16 or 32 wavefronts, 8 or 16 steps per region, schedules
    // around the rates it sustains on such tables (measured: best at
    // 6,000-6,500 GB/s; faster schedules fall behind and lose the order).
    const uint32_t groups[2] = {16, 32};
    const uint32_t gsteps[2] = {8, 16};
    const uint32_t paces[7] = {5750, 6000, 6125, 6250, 6375, 6500, 6750};
    for (uint32_t gi = 0; gi < 2; ++gi) {
        for (uint32_t ki = 0; ki < 2; ++ki) {
            for (uint32_t pi = 0; pi < 7; ++pi) {
                rngx_batch_cfg c{};
                c.values_per_lane = 16;
                c.waves_per_block = 4;
                c.blocks = 0;
                c.use_graph = g.cfg.use_graph;
                c.row_values = 16;
                c.run_items = 0;
                c.per_item = 0;
                c.group = groups[gi];
                c.group_steps = gsteps[ki];
                c.pace_gbs = paces[pi];
                if ((rc = try_cfg(c)))
                    return rc;
            }
        }
    }
    // Confirmation: the four fastest candidates again, each with three
    // times the launches; the fastest there is kept (a schedule just above
    // what a table sustains can time fast once and then fall behind).
    constexpr int kConfirm = RNGX_TUNE_CONFIRM;
    const uint32_t recorded = std::min<uint32_t>(result->n_tried, RNGX_TUNE_MAX);
    int fastest[kConfirm];
    for (int k = 0; k < kConfirm; ++k) {
        fastest[k] = -1;
        for (uint32_t i = 0; i < recorded; ++i) {
            bool taken = false;
            for (int p = 0; p < k; ++p)
                taken = taken || fastest[p] == (int)i;
            if (!taken && (fastest[k] < 0 || result->tried[i].ms < result->tried[fastest[k]].ms))
                fastest[k] = (int)i;
        }
    }
    best = 1e300;
    for (int k = 0; k < kConfirm; ++k) {
        if (fastest[k] < 0)
            continue;
        const rngx_batch_cfg c = result->tried[fastest[k]].cfg;
        if ((rc = batch_stage(g.api_slot, reqs, m, out, out_cap, c.values_per_lane, &total)))
            return rc;
        if ((rc = batch_launch(g.api_slot, c, star, s))) // warm-up (and graph capture)
            return rc;
        RNGX_HIP(hipEventRecord(e0, s));
        for (uint32_t r = 0; r < 3 * reps; ++r)
            if ((rc = batch_launch(g.api_slot, c, star, s)))
                return rc;
        RNGX_HIP(hipEventRecord(e1, s));
        RNGX_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RNGX_HIP(hipEventElapsedTime(&ms, e0, e1));
        result->confirm[k].cfg = c;
        result->confirm[k].ms = (double)ms / (3 * reps);
        if (result->confirm[k].ms < best) {
            best = result->confirm[k].ms;
            result->best = c;
        }
    }
    result->best_ms = best;
    result->best_gbs = (double)total * 8.0 / (best * 1e-3) / 1e9;
    g.cfg = result->best;
    return tune_cache_record_batch(g.cfg, best, m, total);
}
