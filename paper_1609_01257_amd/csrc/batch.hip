// Batched ragged streams in one persistent launch.
//
// Request j names one stream (seed_j, gid_j) and asks for length_j values
// starting at value number offset_j; outputs are packed one request after
// another:  out[base_j + t] = V(seed_j, gid_j, offset_j + t).
//
// Work decomposition. The packed output index space is cut into tiles of
// C = 64 * S values aligned to multiples of C. A work item is one (request,
// tile) pair whose ranges intersect; items are numbered request by request,
// so item -> request is a binary search over the requests' first item
// numbers. A fixed grid of wavefronts takes items in order from an atomic
// counter (items differ in cost: head and tail tiles of a request are
// partial), and every wave leaves the loop when the items run out.
//
// Per item, lane l produces the S values of the tile's l-th sub-range. Its
// starting state comes from GF(2) jump-ahead. The wave first jumps from the
// stream's initial state to the tile's first position with the T^(2^b)
// tables, all lanes at once: lane r holds row r of a jump matrix M and M x
// is one AND, two popcounts and a ballot (x is uniform across the wave).
// Each lane m then places itself m S values further with a lane-spread
// table: T^(m S) z is the XOR of 16 entries, one per nibble of the uniform
// z, and the 64 lanes read 64 consecutive entries (one coalesced load per
// nibble). Each lane then emits R values per round into its own LDS row
// (one 128-byte line for R = 16), and the wave writes the 64 lines back
// with 16-byte stores, 8 lanes per line, so every store instruction covers
// whole lines. LDS and cross-lane operations appear only for this
// bookkeeping.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "internal.h"

namespace rngx {

namespace {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
// Pointers that come from the request table are generic; these casts tell
// the compiler they address global memory, so it emits global (not flat)
// loads and stores: flat operations would also count against the LDS wait
// counter and make every LDS wait stall on outstanding global stores.
typedef __attribute__((address_space(1))) u64x2 g_u64x2;
typedef __attribute__((address_space(1))) uint64_t g_u64;
// The request table is read-only for the whole launch (it is uploaded
// before the kernel starts), so it is read through the constant address
// space: uniform reads (the binary search, a wave's request record) become
// scalar loads, which wait on the scalar counter instead of the vector one
// that the wave's outstanding stores also occupy.
typedef __attribute__((address_space(4))) const BatchReq g_req;
typedef __attribute__((address_space(1))) const uint64_t g_cu64;

// Each round a lane emits R values (R = 8 or 16: a 64- or 128-byte row of
// its own output) into its LDS row of R + 2 words (padding spreads banks).
constexpr int MAX_WAVES_PER_BLOCK = 4;
__host__ __device__ constexpr int lds_row(int R) { return R + 2; }

__device__ __forceinline__ uint64_t wave_matvec(uint64_t row, uint64_t x)
{
    const uint64_t t = row & x;
    const uint32_t pc = __builtin_popcount((uint32_t)t) + __builtin_popcount((uint32_t)(t >> 32));
    return __ballot((pc & 1u) != 0u);
}

// T^k x for a wave-uniform k and x, with pow2 = 64 matrices of 64 rows.
// (Loading several factors' rows ahead of use measured slower.)
__device__ __forceinline__ uint64_t wave_jump(const uint64_t *__restrict__ pow2, uint32_t lane,
                                              uint64_t x, uint64_t k)
{
    while (k) {
        const int b = __builtin_ctzll(k);
        x = wave_matvec(pow2[64 * b + lane], x);
        k &= k - 1;
    }
    return x;
}

// Request of a work item: the last j < m with item_begin[j] <= item (the
// item starts strictly increase from item_begin[0] = 0).
//
// A 64-way search by the whole wave: each round every lane tests one
// candidate and a ballot keeps the chunk that holds the answer (two rounds
// for 4,096 requests). Used when each wave handles one item: it cuts the
// latency before the wave's first store (one wave per S = 128 item: 5.6 ->
// 6.1 TB/s). A persistent wave searches with bisection instead, which runs
// on the scalar unit and measured the same there. (The first round always
// reads the first record; while the records shared a cache line with the
// work counter, that read queued behind every wave's atomic and the
// persistent loop ran three times slower.)
__device__ __forceinline__ uint32_t find_request(g_req *__restrict__ reqs, uint32_t m,
                                                 uint64_t item, uint32_t lane)
{
    uint32_t lo = 0, n = m; // the answer lies in [lo, lo + n)
    while (n > 1) {
        const uint32_t step = (n + 63) / 64;
        const uint32_t off = lane * step;
        const bool le = off < n && reqs[lo + off].item_begin <= item;
        const uint64_t ok = __ballot(le); // a prefix of the lanes, lane 0 always
        const uint32_t k = 63 - __builtin_clzll(ok);
        lo += k * step;
        n = (n - k * step) < step ? (n - k * step) : step;
    }
    return __builtin_amdgcn_readfirstlane(lo); // uniform by construction
}

__device__ __forceinline__ uint32_t bisect_request(g_req *__restrict__ reqs, uint32_t m,
                                                   uint64_t item)
{
    uint32_t lo = 0, hi = m;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (reqs[mid].item_begin <= item)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// A wave-uniform 64-bit value, stated as such to the compiler (its two
// halves read from the first active lane).
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Next work item for the wave: lane 0 bumps the counter with a (vector)
// global atomic and the value is broadcast to the wave.
__device__ __forceinline__ uint64_t next_item(unsigned long long *counter, uint32_t lane,
                                              uint32_t count)
{
    unsigned long long v = 0;
    if (lane == 0)
        v = atomicAdd(counter, (unsigned long long)count);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// y = M x for a lane's own x, M given as 16 tables of 16 entries (entry v of
// table q is M (v << 4q)) held in LDS: the XOR of one lookup per nibble of x.
// Each table spans 128 bytes, so the lanes' lookups never share a bank.
__device__ __forceinline__ uint64_t lane_carry(const uint64_t *__restrict__ tab, uint64_t x)
{
    uint64_t y = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q)
        y ^= tab[16 * q + (uint32_t)((x >> (4 * q)) & 15u)];
    return y;
}

// The word emitted for state x: the state (the paper's generator) or, for the
// scrambled variant, the state times 2685821657736338717 modulo 2^64 (the
// xorshift* multiplier of Vigna, 2016).
template <bool STAR> __device__ __forceinline__ uint64_t out_word(uint64_t x)
{
    return STAR ? x * 2685821657736338717ull : x;
}

// The fields of a request that one work item needs, read once per item.
struct ItemReq {
    uint64_t offset, length, vbase, item_begin, first_tile;
    uint64_t *dst;
    uint32_t gid, mix_low, mix_high, zero_fix;
};

__device__ __forceinline__ ItemReq load_req(g_req *__restrict__ reqs, uint32_t j)
{
    g_req &r = reqs[j];
    ItemReq q;
    q.offset = r.offset;
    q.length = r.length;
    q.vbase = r.vbase;
    q.item_begin = r.item_begin;
    q.first_tile = r.first_tile;
    q.dst = r.dst;
    q.gid = r.gid;
    q.mix_low = r.mix_low;
    q.mix_high = r.mix_high;
    q.zero_fix = r.zero_fix;
    return q;
}

// What a wave does for one work item of request r once r is known: the
// lanes' starting states (from the stream start, or carried from the
// previous tile of the same request), then S values per lane through LDS
// rows and out with whole-line stores. Returns whether the tile was full,
// in which case each lane's state ends S values past its start.
template <int S, int R, bool STAR, bool NT = false>
__device__ __forceinline__ bool process_item(const ItemReq &r, uint64_t item, bool carry,
                                             uint64_t &x, uint64_t *lds,
                                             const uint64_t *carry_tab,
                                             const uint64_t *__restrict__ pow2,
                                             const uint64_t *__restrict__ spread,
                                             g_cu64 *__restrict__ states, uint32_t lane)
{
    constexpr uint64_t C = 64ull * S;
    constexpr int ROUND = R;
    constexpr int LDS_ROW = lds_row(R);
    constexpr uint32_t CPR = R / 2;     // 16-byte chunks per row
    constexpr uint32_t RPI = 64 / CPR;  // rows per store instruction
    const uint64_t B = r.vbase, E = r.vbase + r.length;
    // Output address of virtual index P is obase + P (obase = dst - vbase).
    g_u64 *__restrict__ obase =
        (g_u64 *)(reinterpret_cast<uintptr_t>(r.dst) - B * sizeof(uint64_t));
    const uint64_t T0 = (r.first_tile + (item - r.item_begin)) * C;

    if (carry) {
        x = lane_carry(carry_tab, x);
    } else {
        const uint64_t q0 = T0 > B ? T0 : B;
        // State at q0, then each active lane's first position.
        SeedMix mix;
        mix.mix_low = r.mix_low;
        mix.mix_high = r.mix_high;
        mix.zero_fix = r.zero_fix;
        const uint64_t x0 = states ? states[r.gid] : init_state(mix, r.gid);
        const uint64_t xq0 = wave_jump(pow2, lane, x0, r.offset + (q0 - B));
        // Lanes from b on start at T0 + l S = (T0 + b S) + (l - b) S: with
        // z the state at T0 + b S, lane l takes T^((l - b) S) z from the
        // spread table. If the request starts inside lane l0's range, that
        // lane takes the state at q0 itself and b = l0 + 1.
        uint32_t b = 0, l0 = 64;
        uint64_t z = xq0;
        if (q0 != T0) {
            const uint32_t d = (uint32_t)(q0 - T0); // < C
            const uint32_t rem = d % (uint32_t)S;
            b = d / (uint32_t)S;
            if (rem != 0) {
                l0 = b++;
                if (b < 64)
                    z = wave_jump(pow2, lane, xq0, (uint64_t)S - rem);
            }
        }
        x = 0;
        if (lane >= b) {
            const uint64_t *__restrict__ col = spread + (lane - b);
            uint64_t e[16];
#pragma unroll
            for (int q = 0; q < 16; ++q)
                e[q] = col[(16u * q + (uint32_t)((z >> (4 * q)) & 15u)) * 64u];
#pragma unroll
            for (int q = 0; q < 16; ++q)
                x ^= e[q];
        }
        if (lane == l0)
            x = xq0;
    }

    const bool full = T0 >= B && T0 + C <= E;
    const uint64_t my0 = T0 + (uint64_t)lane * S;
    for (uint32_t rd = 0; rd < (uint32_t)S / ROUND; ++rd) {
        const uint64_t p0 = my0 + (uint64_t)rd * ROUND;
        if (full) {
#pragma unroll
            for (int s = 0; s < ROUND; ++s) {
                lds[lane * LDS_ROW + s] = out_word<STAR>(x);
                x = xs_step(x);
            }
        } else {
#pragma unroll
            for (int s = 0; s < ROUND; ++s) {
                const uint64_t P = p0 + s;
                if (P >= B && P < E) {
                    lds[lane * LDS_ROW + s] = out_word<STAR>(x);
                    x = xs_step(x);
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // Lane l of store instruction i writes 16 bytes of row RPI*i + l/CPR:
        // CPR lanes cover one row, i.e. one whole 64- or 128-byte segment.
        const uint32_t ch = lane % CPR;
        if (full) {
            u64x2 v[CPR];
#pragma unroll
            for (uint32_t i = 0; i < CPR; ++i) {
                const uint32_t row = RPI * i + lane / CPR;
                v[i] = *reinterpret_cast<const u64x2 *>(&lds[row * LDS_ROW + 2u * ch]);
            }
            // Wave-uniform tile base plus a 32-bit lane offset (a tile is at
            // most 512 KiB).
            g_u64 *__restrict__ tile = obase + T0;
#pragma unroll
            for (uint32_t i = 0; i < CPR; ++i) {
                const uint32_t row = RPI * i + lane / CPR;
                const uint32_t off = row * (uint32_t)S + rd * (uint32_t)ROUND + 2u * ch;
                if (NT)
                    __builtin_nontemporal_store(v[i], (g_u64x2 *)(tile + off));
                else
                    *(g_u64x2 *)(tile + off) = v[i];
            }
        } else {
#pragma unroll
            for (uint32_t i = 0; i < CPR; ++i) {
                const uint32_t row = RPI * i + lane / CPR;
                const uint64_t P = T0 + (uint64_t)row * S + (uint64_t)rd * ROUND + 2u * ch;
                const u64x2 v = *reinterpret_cast<const u64x2 *>(&lds[row * LDS_ROW + 2u * ch]);
                const bool v0 = P >= B && P < E;
                const bool v1 = P + 1 >= B && P + 1 < E;
                if (v0 && v1)
                    *(g_u64x2 *)(obase + P) = v;
                else if (v0)
                    obase[P] = v.x;
                else if (v1)
                    obase[P + 1] = v.y;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    return full;
}

template <int S, int R, bool STAR>
__global__ __launch_bounds__(256) void batch_kernel(const BatchDesc *__restrict__ desc,
                                                    const uint64_t *__restrict__ pow2,
                                                    const uint64_t *__restrict__ spread,
                                                    const uint64_t *__restrict__ carry_nib,
                                                    uint32_t run_items, uint32_t per_item)
{
    constexpr int LDS_ROW = lds_row(R);
    // Dynamic LDS: 64 * LDS_ROW u64 per wave, then the carry table (rows
    // first keeps row addresses small enough for the LDS offset fields).
    extern __shared__ uint64_t lds_dyn[];
    const uint32_t lane = threadIdx.x & 63u;
    // Wave index, made provably uniform so item bookkeeping runs on the
    // scalar unit and the request table is read with scalar loads.
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t *carry_tab = lds_dyn + (size_t)(blockDim.x >> 6) * 64 * LDS_ROW;
    uint64_t *lds = lds_dyn + (size_t)wid * 64 * LDS_ROW;
    if (!per_item) {
        // Only runs carry state; the barrier is uniform (per_item is).
        for (uint32_t i = threadIdx.x; i < (uint32_t)kCarryTable; i += blockDim.x)
            carry_tab[i] = carry_nib[i];
        __syncthreads();
    }

    const uint64_t n_items = desc->n_items;
    const uint32_t m = desc->m;
    g_req *__restrict__ reqs = (g_req *)desc->reqs;
    g_cu64 *__restrict__ states = (g_cu64 *)desc->states;
    unsigned long long *counter =
        reinterpret_cast<unsigned long long *>(const_cast<uint64_t *>(&desc->next_item));

    // A wave takes runs of `run_items` consecutive items. While it stays on
    // one request and the previous tile was full, every lane's state is
    // already S values past its previous start and needs C - S more steps
    // (one per-lane product with T^(C-S)): no search or jump.
    // Runs shrink towards the end of the batch (guided self-scheduling: at
    // most the items left, as last seen, over twice the number of waves), so
    // the last runs taken do not leave a long tail.
    const uint64_t n_waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    uint64_t item = 0, run_end = 0, req_end = 0, seen = 0;
    uint32_t lo = 0;
    bool carry = false;
    uint64_t x = 0;
    if (per_item) {
        // One wave per work item: the grid covers the items exactly once.
        item = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wid;
        if (item >= n_items)
            return;
        run_end = item + 1;
    }
    for (;;) {
        item = uniform64(item);
        if (item >= run_end) {
            if (per_item)
                break;
            uint64_t want = 1;
            if (run_items > 1) {
                const uint64_t share = (n_items > seen ? n_items - seen : 0) / (2 * n_waves);
                want = share < 1 ? 1 : (share < run_items ? share : run_items);
            }
            item = next_item(counter, lane, (uint32_t)want);
            if (item >= n_items)
                break;
            seen = item + want;
            run_end = seen < n_items ? seen : n_items;
            carry = false;
        }
        if (!carry) {
            lo = per_item ? find_request(reqs, m, item, lane) : bisect_request(reqs, m, item);
            lo = __builtin_amdgcn_readfirstlane(lo);
            req_end = uniform64(lo + 1 < m ? (uint64_t)reqs[lo + 1].item_begin : n_items);
        }
        const ItemReq r = load_req(reqs, lo);
        const bool full = process_item<S, R, STAR>(r, item, carry, x, lds, carry_tab, pow2,
                                                   spread, states, lane);
        // Lane l now holds the state at T0 + l*S + S when the tile was full.
        // Every quantity of this loop is the same in all lanes; saying so
        // keeps the bookkeeping, the request search and the record loads on
        // the scalar unit (otherwise the carried flag makes the compiler
        // treat the next search as divergent, with per-lane vector loads).
        ++item;
        carry = __builtin_amdgcn_readfirstlane(
                    (uint32_t)(full && item < run_end && item < req_end)) != 0;
    }
}

// A full tile at virtual index T0 of a request whose output index 0 is at
// obase[vbase]: lane l holds the state at T0 + l*S; S values per lane
// through LDS rows, whole-line stores. Same stores as process_item's full
// path.
template <int S, int R, bool STAR, bool NT>
__device__ __forceinline__ void emit_full_tile(uint64_t &x, uint64_t *lds, g_u64 *__restrict__ tile,
                                               uint32_t lane)
{
    constexpr int ROUND = R;
    constexpr int LDS_ROW = lds_row(R);
    constexpr uint32_t CPR = R / 2;
    constexpr uint32_t RPI = 64 / CPR;
    for (uint32_t rd = 0; rd < (uint32_t)S / ROUND; ++rd) {
#pragma unroll
        for (int s = 0; s < ROUND; ++s) {
            lds[lane * LDS_ROW + s] = out_word<STAR>(x);
            x = xs_step(x);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t ch = lane % CPR;
        u64x2 v[CPR];
#pragma unroll
        for (uint32_t i = 0; i < CPR; ++i) {
            const uint32_t row = RPI * i + lane / CPR;
            v[i] = *reinterpret_cast<const u64x2 *>(&lds[row * LDS_ROW + 2u * ch]);
        }
#pragma unroll
        for (uint32_t i = 0; i < CPR; ++i) {
            const uint32_t row = RPI * i + lane / CPR;
            const uint32_t off = row * (uint32_t)S + rd * (uint32_t)ROUND + 2u * ch;
            if (NT)
                __builtin_nontemporal_store(v[i], (g_u64x2 *)(tile + off));
            else
                *(g_u64x2 *)(tile + off) = v[i];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Wait (bounded) until the device's constant-rate clock reaches `due`: at
// most about 2^16 polls of about 100 ns, so a wait ends whatever the clock
// does. Uniform across the wavefront (a scalar clock read).
__device__ __forceinline__ void wait_clock(uint64_t due)
{
    uint32_t polls = 0;
    while (__builtin_amdgcn_s_memrealtime() < due && ++polls < (1u << 16))
        __builtin_amdgcn_s_sleep(2);
}

// The grouped order (rngx_batch_cfg.group). The grid's wavefronts form
// groups of `group`; the work items are cut into regions of group * steps
// consecutive items, group q takes regions q, q + Q, ... (Q groups), and at
// step s of a region its wavefront j takes item s * group + j. A group's
// wavefronts thus write neighbouring tiles and move through the region
// together: at any time the grid writes a few dense windows instead of one
// scattered tile per wavefront. Within a request a wavefront's next item is
// `group` tiles on, so each lane carries its state group * C - S values on
// with one nibble-table product (`group_nib`, in LDS); it jumps from the
// stream's start only at a region's or a request's first item. With
// delta256 != 0 every wavefront takes its step k no earlier than its start
// time + k * delta256 / 256 clock ticks.
template <int S, int R, bool STAR>
__global__ __launch_bounds__(256) void batch_group_kernel(const BatchDesc *__restrict__ desc,
                                                          const uint64_t *__restrict__ pow2,
                                                          const uint64_t *__restrict__ spread,
                                                          const uint64_t *__restrict__ group_nib,
                                                          uint32_t group, uint32_t steps,
                                                          uint64_t delta256)
{
    constexpr int LDS_ROW = lds_row(R);
    extern __shared__ uint64_t lds_dyn[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t *stride_tab = lds_dyn + (size_t)(blockDim.x >> 6) * 64 * LDS_ROW;
    uint64_t *lds = lds_dyn + (size_t)wid * 64 * LDS_ROW;
    for (uint32_t i = threadIdx.x; i < (uint32_t)kCarryTable; i += blockDim.x)
        stride_tab[i] = group_nib[i];
    __syncthreads();

    const uint64_t n_items = desc->n_items;
    const uint32_t m = desc->m;
    g_req *__restrict__ reqs = (g_req *)desc->reqs;
    g_cu64 *__restrict__ states = (g_cu64 *)desc->states;
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wid;
    const uint64_t n_groups = (uint64_t)gridDim.x * (blockDim.x >> 6) / group;
    const uint64_t q = wave / group, j = wave % group;
    if (q >= n_groups)
        return;
    const uint64_t per_region = (uint64_t)group * steps;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    constexpr uint64_t C = 64ull * S;
    uint64_t sched = 0, x = 0, req_end = 0;
    uint32_t lo = 0;
    // The current request while carrying: its last tile start T0, its end
    // E (virtual indices) and its output base address (output of virtual
    // index P at obase + P).
    uint64_t cur_T0 = 0, cur_E = 0, cur_obase = 0;
    for (uint64_t reg = q; reg * per_region < n_items; reg += n_groups) {
        bool carry = false;
        for (uint32_t st = 0; st < steps; ++st) {
            const uint64_t item = uniform64(reg * per_region + (uint64_t)st * group + j);
            if (item >= n_items)
                break; // the rest of the region lies further on
            if (delta256) {
                wait_clock(t0 + (sched >> 8));
                sched += delta256;
            }
            if (carry && cur_T0 + (uint64_t)group * C + C <= cur_E) {
                // A full tile `group` tiles on in the same request.
                cur_T0 = uniform64(cur_T0 + (uint64_t)group * C);
                x = lane_carry(stride_tab, x);
                emit_full_tile<S, R, STAR, true>(
                    x, lds, reinterpret_cast<g_u64 *>(cur_obase) + cur_T0, lane);
                carry = __builtin_amdgcn_readfirstlane(
                            (uint32_t)(item + group < req_end)) != 0;
                continue;
            }
            if (!carry) {
                lo = __builtin_amdgcn_readfirstlane(bisect_request(reqs, m, item));
                req_end = uniform64(lo + 1 < m ? (uint64_t)reqs[lo + 1].item_begin : n_items);
            }
            const ItemReq r = load_req(reqs, lo);
            cur_T0 = uniform64((r.first_tile + (item - r.item_begin)) * C);
            cur_E = uniform64(r.vbase + r.length);
            cur_obase = uniform64(reinterpret_cast<uintptr_t>(r.dst) - r.vbase * sizeof(uint64_t));
            const bool full = process_item<S, R, STAR, true>(r, item, carry, x, lds, stride_tab,
                                                             pow2, spread, states, lane);
            // Lane l holds the state at T0 + l*S + S when the tile was full;
            // the wave's next item is `group` tiles on if it is still in
            // this request.
            carry = __builtin_amdgcn_readfirstlane(
                        (uint32_t)(full && item + group < req_end)) != 0;
        }
    }
}

// A batch of at most kSmallReqs requests with its table in the kernel's
// arguments: one wave per work item, no table upload before the launch.
template <int S, int R, bool STAR>
__global__ __launch_bounds__(256) void batch_small_kernel(const SmallTable t,
                                                          const uint64_t *__restrict__ pow2,
                                                          const uint64_t *__restrict__ spread)
{
    constexpr int LDS_ROW = lds_row(R);
    extern __shared__ uint64_t lds_dyn[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint64_t *lds = lds_dyn + (size_t)wid * 64 * LDS_ROW;
    const uint64_t item = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wid;
    if (item >= t.desc.n_items)
        return;
    // The last request whose first item is at most this item (m is small).
    uint32_t lo = 0;
    for (uint32_t j = 1; j < t.desc.m; ++j)
        if (t.reqs[j].item_begin <= item)
            lo = j;
    const BatchReq &q = t.reqs[lo];
    ItemReq r;
    r.offset = q.offset;
    r.length = q.length;
    r.vbase = q.vbase;
    r.item_begin = q.item_begin;
    r.first_tile = q.first_tile;
    r.dst = q.dst;
    r.gid = q.gid;
    r.mix_low = q.mix_low;
    r.mix_high = q.mix_high;
    r.zero_fix = q.zero_fix;
    uint64_t x = 0;
    (void)process_item<S, R, STAR>(r, item, false, x, lds, nullptr, pow2, spread,
                                   (g_cu64 *)t.desc.states, lane);
}

template <int S, int R, bool STAR>
hipError_t launch_group_t(const BatchDesc *desc, const BatchTables &t, const rngx_batch_cfg &c,
                          size_t lds_bytes, hipStream_t s)
{
    uint64_t delta256 = 0;
    if (c.pace_gbs) {
        // One step: every wavefront of the grid writes one tile.
        const double step_bytes = (double)c.blocks * c.waves_per_block * 64.0 * S * 8.0;
        delta256 = (uint64_t)(step_bytes / (c.pace_gbs * 1e9) * t.clock_khz * 1e3 * 256.0);
    }
    batch_group_kernel<S, R, STAR><<<dim3(c.blocks), dim3(64 * c.waves_per_block), lds_bytes, s>>>(
        desc, t.pow2, t.spread, t.group_nib, c.group, c.group_steps, delta256);
    return hipGetLastError();
}

template <int S, bool STAR>
hipError_t launch_batch_s(const BatchDesc *desc, const BatchTables &t, const rngx_batch_cfg &c,
                          hipStream_t s)
{
    const size_t lds_bytes =
        (kCarryTable + (size_t)c.waves_per_block * 64 * lds_row(c.row_values)) * sizeof(uint64_t);
    if (c.group)
        return c.row_values == 8 ? launch_group_t<S, 8, STAR>(desc, t, c, lds_bytes, s)
                                 : launch_group_t<S, 16, STAR>(desc, t, c, lds_bytes, s);
    const uint32_t run = c.run_items ? c.run_items : 1;
    if (c.row_values == 8)
        batch_kernel<S, 8, STAR><<<dim3(c.blocks), dim3(64 * c.waves_per_block), lds_bytes, s>>>(
            desc, t.pow2, t.spread, t.carry_nib, run, c.per_item);
    else
        batch_kernel<S, 16, STAR><<<dim3(c.blocks), dim3(64 * c.waves_per_block), lds_bytes, s>>>(
            desc, t.pow2, t.spread, t.carry_nib, run, c.per_item);
    return hipGetLastError();
}

template <int S, bool STAR>
hipError_t launch_batch_small_s(const SmallTable &tab, const BatchTables &t,
                                const rngx_batch_cfg &c, hipStream_t s)
{
    const size_t lds_bytes = (size_t)c.waves_per_block * 64 * lds_row(c.row_values) * 8;
    if (c.row_values == 8)
        batch_small_kernel<S, 8, STAR>
            <<<dim3(c.blocks), dim3(64 * c.waves_per_block), lds_bytes, s>>>(tab, t.pow2, t.spread);
    else
        batch_small_kernel<S, 16, STAR>
            <<<dim3(c.blocks), dim3(64 * c.waves_per_block), lds_bytes, s>>>(tab, t.pow2, t.spread);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void checksum_kernel(const uint64_t *__restrict__ d, uint64_t n,
                                                       unsigned long long *acc)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        s += d[i] * (2 * i + 1);
    for (int off = 32; off > 0; off >>= 1)
        s += __shfl_xor(s, off);
    if ((threadIdx.x & 63u) == 0)
        atomicAdd(acc, s);
}

} // namespace

hipError_t launch_checksum(const uint64_t *data, uint64_t n, uint64_t *acc, hipStream_t s)
{
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks == 0)
        blocks = 1;
    checksum_kernel<<<dim3((uint32_t)blocks), dim3(256), 0, s>>>(
        data, n, reinterpret_cast<unsigned long long *>(acc));
    return hipGetLastError();
}

bool batch_cfg_valid(const rngx_batch_cfg &c)
{
    const bool s_ok = c.values_per_lane == 8 || c.values_per_lane == 16 ||
                      c.values_per_lane == 32 || c.values_per_lane == 64 ||
                      c.values_per_lane == 128 || c.values_per_lane == 256 ||
                      c.values_per_lane == 512 || c.values_per_lane == 1024;
    const bool base = s_ok && c.waves_per_block >= 1 &&
                      c.waves_per_block <= MAX_WAVES_PER_BLOCK && c.blocks <= 65536 &&
                      c.use_graph <= 1 && (c.row_values == 8 || c.row_values == 16) &&
                      c.row_values <= c.values_per_lane && c.run_items <= 64 && c.per_item <= 1;
    if (!base)
        return false;
    if (c.group == 0)
        return c.group_steps == 0 && c.pace_gbs == 0;
    return batch_group_index(c.group) >= 0 && c.group % c.waves_per_block == 0 &&
           c.group_steps >= 1 && c.group_steps <= 256 && c.per_item == 0 &&
           (c.pace_gbs == 0 || (c.pace_gbs >= 1000 && c.pace_gbs <= 20000));
}

hipError_t batch_group_occupancy(const rngx_batch_cfg &c, int *blocks_per_cu)
{
    const size_t lds_bytes =
        (kCarryTable + (size_t)c.waves_per_block * 64 * lds_row(c.row_values)) * sizeof(uint64_t);
    const int threads = (int)(64 * c.waves_per_block);
    // Every S and star variant shares the resource use of its row width
    // closely enough for the grid size; the S = 16 kernels stand for all.
    return c.row_values == 8
               ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     blocks_per_cu, batch_group_kernel<16, 8, false>, threads, lds_bytes)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     blocks_per_cu, batch_group_kernel<16, 16, false>, threads, lds_bytes);
}

template <bool STAR>
hipError_t launch_batch_star(const rngx_batch_cfg &cfg, const BatchDesc *desc,
                             const BatchTables &t, hipStream_t s)
{
    switch (cfg.values_per_lane) {
    case 8: return launch_batch_s<8, STAR>(desc, t, cfg, s);
    case 16: return launch_batch_s<16, STAR>(desc, t, cfg, s);
    case 32: return launch_batch_s<32, STAR>(desc, t, cfg, s);
    case 64: return launch_batch_s<64, STAR>(desc, t, cfg, s);
    case 128: return launch_batch_s<128, STAR>(desc, t, cfg, s);
    case 256: return launch_batch_s<256, STAR>(desc, t, cfg, s);
    case 512: return launch_batch_s<512, STAR>(desc, t, cfg, s);
    default: return launch_batch_s<1024, STAR>(desc, t, cfg, s);
    }
}

template <bool STAR>
hipError_t launch_batch_small_star(const rngx_batch_cfg &cfg, const SmallTable &tab,
                                   const BatchTables &t, hipStream_t s)
{
    switch (cfg.values_per_lane) {
    case 8: return launch_batch_small_s<8, STAR>(tab, t, cfg, s);
    case 16: return launch_batch_small_s<16, STAR>(tab, t, cfg, s);
    case 32: return launch_batch_small_s<32, STAR>(tab, t, cfg, s);
    case 64: return launch_batch_small_s<64, STAR>(tab, t, cfg, s);
    case 128: return launch_batch_small_s<128, STAR>(tab, t, cfg, s);
    case 256: return launch_batch_small_s<256, STAR>(tab, t, cfg, s);
    case 512: return launch_batch_small_s<512, STAR>(tab, t, cfg, s);
    default: return launch_batch_small_s<1024, STAR>(tab, t, cfg, s);
    }
}

hipError_t launch_batch(const rngx_batch_cfg &cfg, const BatchDesc *desc, const BatchTables &t,
                        bool star, hipStream_t s)
{
    return star ? launch_batch_star<true>(cfg, desc, t, s)
                : launch_batch_star<false>(cfg, desc, t, s);
}

hipError_t launch_batch_small(const rngx_batch_cfg &cfg, const SmallTable &tab,
                              const BatchTables &t, bool star, hipStream_t s)
{
    return star ? launch_batch_small_star<true>(cfg, tab, t, s)
                : launch_batch_small_star<false>(cfg, tab, t, s);
}

} // namespace rngx
