// Seeding and plain-generation kernels for gfx950 (CDNA4, wave64).
//
// init: one state per work-item, state[g] = H(seed, g) (Listing S4).
// gen:  a persistent loop per lane. The lane loads its states once, then for
//       every iteration k stores them to row k of the iteration-major output
//       and advances them one xorshift step (Listing S5), and finally writes
//       them back. The paper's kernel reads and writes 16 bytes of state per
//       value per launch; here state traffic is 16 bytes per work-item per
//       call, and each value costs only its 8 (or 4) output bytes.
//
// Store layout: a wavefront owns 64 * V consecutive work-items (V = 2*P for
// 64-bit output, 4*P for 32-bit), split into P "chunk columns". In column p,
// lane l owns the 16 bytes at work-items [base + p*64*E + l*E, +E), E = 16 /
// sizeof(T). So every store instruction of the wave writes one contiguous
// 1 KiB line-aligned span (global_store_dwordx4 from all 64 lanes) whenever
// the row start is 16-byte aligned. No LDS and no cross-lane traffic.
#include <atomic>

#include "internal.h"

namespace rngx {
namespace {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void init_kernel(uint64_t *__restrict__ state, uint32_t n,
                                                   SeedMix mix)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += stride)
        state[g] = init_state(mix, (uint32_t)g);
}

// The word emitted for state x. The paper's generator emits the state (its
// low half for 32-bit output). The scrambled variant emits the state times
// 2685821657736338717 modulo 2^64 (the xorshift* multiplier of Vigna, 2016),
// its high half for 32-bit output; the state sequence is the same.
constexpr uint64_t kStarMultiplier = 2685821657736338717ull;
template <typename T, bool STAR> __device__ __forceinline__ T emit(uint64_t x);
template <> __device__ __forceinline__ uint64_t emit<uint64_t, false>(uint64_t x) { return x; }
template <> __device__ __forceinline__ uint32_t emit<uint32_t, false>(uint64_t x)
{
    return (uint32_t)x;
}
template <> __device__ __forceinline__ uint64_t emit<uint64_t, true>(uint64_t x)
{
    return x * kStarMultiplier;
}
template <> __device__ __forceinline__ uint32_t emit<uint32_t, true>(uint64_t x)
{
    return (uint32_t)((x * kStarMultiplier) >> 32);
}

template <typename T> struct Vec16;
template <> struct Vec16<uint64_t> {
    static constexpr int E = 2;
    typedef u64x2 type;
    template <bool STAR> __device__ static __forceinline__ type pack(const uint64_t *x)
    {
        return type{emit<uint64_t, STAR>(x[0]), emit<uint64_t, STAR>(x[1])};
    }
};
template <> struct Vec16<uint32_t> {
    static constexpr int E = 4;
    typedef u32x4 type;
    template <bool STAR> __device__ static __forceinline__ type pack(const uint64_t *x)
    {
        return type{emit<uint32_t, STAR>(x[0]), emit<uint32_t, STAR>(x[1]),
                    emit<uint32_t, STAR>(x[2]), emit<uint32_t, STAR>(x[3])};
    }
};

template <bool NT, typename VT> __device__ __forceinline__ void store16(VT *p, VT v)
{
    if (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Wait (bounded) until the device's constant-rate clock reaches `due`.
// Uniform across the wavefront: the clock is read by a scalar instruction.
__device__ __forceinline__ void wait_until(uint64_t due)
{
    // At most about 2^16 polls of about 100 ns: a wait ends even if the
    // schedule were far ahead of the clock.
    uint32_t polls = 0;
    while (__builtin_amdgcn_s_memrealtime() < due && ++polls < (1u << 16))
        __builtin_amdgcn_s_sleep(2);
}

// One complete wavefront: its 64*P*E work-items starting at wbase, all
// iterations. PACED: iteration k is written no earlier than
// t0 + ((sched + k * delta256) >> 8) clock ticks.
template <typename T, int P, bool NT, bool ALIGNED, bool STAR, bool PACED>
__device__ __forceinline__ void full_wave(uint64_t *__restrict__ state, uint32_t n,
                                          uint32_t iters, T *__restrict__ out, uint64_t wbase,
                                          uint32_t lane, uint64_t t0, uint64_t sched,
                                          uint64_t delta256)
{
    typedef Vec16<T> VT;
    constexpr int E = VT::E;
    uint64_t x[P][E];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint64_t g = wbase + (uint64_t)p * 64 * E + (uint64_t)lane * E;
#pragma unroll
        for (int e = 0; e < E; ++e)
            x[p][e] = state[g + e];
    }
    for (uint32_t k = 0; k < iters; ++k) {
        if (PACED) {
            wait_until(t0 + (sched >> 8));
            sched += delta256;
        }
        T *row = out + (size_t)k * n;
        const bool al = ALIGNED || ((reinterpret_cast<uintptr_t>(row) & 15u) == 0);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint64_t g = wbase + (uint64_t)p * 64 * E + (uint64_t)lane * E;
            if (al) {
                store16<NT>(reinterpret_cast<typename VT::type *>(row + g),
                            VT::template pack<STAR>(x[p]));
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e)
                    row[g + e] = emit<T, STAR>(x[p][e]);
            }
#pragma unroll
            for (int e = 0; e < E; ++e)
                x[p][e] = xs_step(x[p][e]);
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint64_t g = wbase + (uint64_t)p * 64 * E + (uint64_t)lane * E;
#pragma unroll
        for (int e = 0; e < E; ++e)
            state[g + e] = x[p][e];
    }
}

// The last, partial wavefront: element-wise guarded (the paper's
// gid < nseeds test).
template <typename T, int P, bool STAR>
__device__ __forceinline__ void partial_wave(uint64_t *__restrict__ state, uint32_t n,
                                             uint32_t iters, T *__restrict__ out, uint64_t wbase,
                                             uint32_t lane)
{
    constexpr int E = Vec16<T>::E;
    uint64_t x[P][E];
    uint32_t cnt[P];
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint64_t g = wbase + (uint64_t)p * 64 * E + (uint64_t)lane * E;
        cnt[p] = g >= n ? 0u : (uint32_t)((n - g) < (uint64_t)E ? (n - g) : E);
#pragma unroll
        for (int e = 0; e < E; ++e)
            x[p][e] = (uint32_t)e < cnt[p] ? state[g + e] : 0u;
    }
    for (uint32_t k = 0; k < iters; ++k) {
        T *row = out + (size_t)k * n;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint64_t g = wbase + (uint64_t)p * 64 * E + (uint64_t)lane * E;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if ((uint32_t)e < cnt[p])
                    row[g + e] = emit<T, STAR>(x[p][e]);
                x[p][e] = xs_step(x[p][e]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
        const uint64_t g = wbase + (uint64_t)p * 64 * E + (uint64_t)lane * E;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if ((uint32_t)e < cnt[p])
                state[g + e] = x[p][e];
    }
}

// P chunk columns per lane; NT: non-temporal stores; ALIGNED: every row
// start is 16-byte aligned (out 16-byte aligned and n*sizeof(T) % 16 == 0).
template <typename T, int P, bool NT, bool ALIGNED, bool STAR>
__global__ __launch_bounds__(1024) void gen_kernel(uint64_t *__restrict__ state, uint32_t n,
                                                   uint32_t iters, T *__restrict__ out)
{
    constexpr uint64_t WAVE_ITEMS = 64ull * P * Vec16<T>::E;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t wbase = wave * WAVE_ITEMS;
    if (wbase >= n)
        return;
    if (wbase + WAVE_ITEMS <= n)
        full_wave<T, P, NT, ALIGNED, STAR, false>(state, n, iters, out, wbase, lane, 0, 0, 0);
    else
        partial_wave<T, P, STAR>(state, n, iters, out, wbase, lane);
}

// The scheduled launch: a persistent grid of gridDim.x blocks, all resident
// at once, walks strips of columns; in strip s, block b owns the columns of
// block s * gridDim.x + b of the unscheduled launch. Every wavefront keeps
// to one row schedule from its own start t0 (its first clock reading):
// iteration k of strip s is written no earlier than
// t0 + (s * iters + k) * delta256 / 256 clock ticks, so the wavefronts write
// near the same row instead of drifting apart. (Measured on MI355X: one
// start time shared by the whole grid, the first wavefront's, ran 3-20 %
// slower at 2^20-2^24 states and the same at 2^26.) Rows are 16-byte
// aligned (the launcher checks it).
template <typename T, int P, bool NT, bool STAR>
__global__ __launch_bounds__(1024) void gen_paced_kernel(uint64_t *__restrict__ state, uint32_t n,
                                                         uint32_t iters, T *__restrict__ out,
                                                         uint32_t nstrips, uint64_t delta256)
{
    constexpr uint64_t WAVE_ITEMS = 64ull * P * Vec16<T>::E;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves_per_block = blockDim.x >> 6;
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    for (uint32_t s = 0; s < nstrips; ++s) {
        const uint64_t wave =
            ((uint64_t)s * gridDim.x + blockIdx.x) * waves_per_block + (threadIdx.x >> 6);
        const uint64_t wbase = wave * WAVE_ITEMS;
        if (wbase >= n)
            return; // later strips lie further right
        if (wbase + WAVE_ITEMS > n) {
            partial_wave<T, P, STAR>(state, n, iters, out, wbase, lane);
            return; // the last wavefront of the launch
        }
        full_wave<T, P, NT, true, STAR, true>(state, n, iters, out, wbase, lane, t0,
                                              (uint64_t)s * iters * delta256, delta256);
    }
}

template <typename T, int P, bool NT, bool AL, bool STAR>
hipError_t launch_gen_t(uint32_t block, uint64_t *state, uint32_t n, uint32_t iters, T *out,
                        hipStream_t s)
{
    constexpr uint64_t WAVE_ITEMS = 64ull * P * Vec16<T>::E;
    const uint64_t waves = (n + WAVE_ITEMS - 1) / WAVE_ITEMS;
    const uint64_t blocks = (waves * 64 + block - 1) / block;
    gen_kernel<T, P, NT, AL, STAR>
        <<<dim3((uint32_t)blocks), dim3(block), 0, s>>>(state, n, iters, out);
    return hipGetLastError();
}

// The scheduled launch: grid = every block that fits on the device at once
// (at most the blocks the columns need); the schedule's step is the time
// the grid's share of a row (blocks x block x 16 x P bytes) takes at
// pace_gbs, in ticks of the device's constant-rate clock, times 256.
template <typename T, int P, bool NT, bool STAR>
hipError_t launch_paced_t(uint32_t block, uint32_t pace_gbs, uint64_t *state, uint32_t n,
                          uint32_t iters, T *out, hipStream_t s)
{
    constexpr uint64_t WAVE_ITEMS = 64ull * P * Vec16<T>::E;
    // Device attributes and this kernel's occupancy at `block`, cached per
    // device (devices beyond the table query every launch).
    constexpr int kDevs = 16;
    static std::atomic<int> cached_occ[kDevs][16] = {};
    static std::atomic<int> cached_cus[kDevs] = {}, cached_khz[kDevs] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    const bool cacheable = dev >= 0 && dev < kDevs;
    const int bi = (int)(block / 64) - 1; // block 64..1024
    int cus = cacheable ? cached_cus[dev].load(std::memory_order_relaxed) : 0;
    int clock_khz = cacheable ? cached_khz[dev].load(std::memory_order_relaxed) : 0;
    int occ = cacheable ? cached_occ[dev][bi].load(std::memory_order_relaxed) : 0;
    if (cus <= 0 || clock_khz <= 0 || occ <= 0) {
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeWallClockRate, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, gen_paced_kernel<T, P, NT, STAR>, (int)block, 0);
        if (e != hipSuccess)
            return e;
        cus = cus > 0 ? cus : 1;
        clock_khz = clock_khz > 0 ? clock_khz : 100000;
        occ = occ > 0 ? occ : 1;
        if (cacheable) {
            cached_cus[dev].store(cus, std::memory_order_relaxed);
            cached_khz[dev].store(clock_khz, std::memory_order_relaxed);
            cached_occ[dev][bi].store(occ, std::memory_order_relaxed);
        }
    }
    const uint64_t waves = (n + WAVE_ITEMS - 1) / WAVE_ITEMS;
    const uint64_t need = (waves * 64 + block - 1) / block;
    uint64_t grid = (uint64_t)occ * (uint64_t)cus;
    if (grid > need)
        grid = need;
    const uint64_t nstrips = (need + grid - 1) / grid;
    const double row_bytes = (double)grid * block * 16.0 * P;
    const double ticks = row_bytes / (pace_gbs * 1e9) * clock_khz * 1e3;
    const uint64_t delta256 = (uint64_t)(ticks * 256.0);
    gen_paced_kernel<T, P, NT, STAR><<<dim3((uint32_t)grid), dim3(block), 0, s>>>(
        state, n, iters, out, (uint32_t)nstrips, delta256);
    return hipGetLastError();
}

template <typename T, int P, bool STAR>
hipError_t launch_gen_p(const rngx_launch &cfg, bool al, uint64_t *state, uint32_t n,
                        uint32_t iters, T *out, hipStream_t s)
{
    if (cfg.pace_gbs && al && iters >= 2)
        return cfg.nontemporal
                   ? launch_paced_t<T, P, true, STAR>(cfg.block, cfg.pace_gbs, state, n, iters,
                                                      out, s)
                   : launch_paced_t<T, P, false, STAR>(cfg.block, cfg.pace_gbs, state, n, iters,
                                                       out, s);
    if (cfg.nontemporal)
        return al ? launch_gen_t<T, P, true, true, STAR>(cfg.block, state, n, iters, out, s)
                  : launch_gen_t<T, P, true, false, STAR>(cfg.block, state, n, iters, out, s);
    return al ? launch_gen_t<T, P, false, true, STAR>(cfg.block, state, n, iters, out, s)
              : launch_gen_t<T, P, false, false, STAR>(cfg.block, state, n, iters, out, s);
}

template <typename T, bool STAR>
hipError_t launch_gen_typed(const rngx_launch &cfg, uint64_t *state, uint32_t n, uint32_t iters,
                            T *out, hipStream_t s)
{
    const bool al = (reinterpret_cast<uintptr_t>(out) & 15u) == 0 &&
                    ((uint64_t)n * sizeof(T)) % 16u == 0;
    switch (cfg.chunks) {
    case 1: return launch_gen_p<T, 1, STAR>(cfg, al, state, n, iters, out, s);
    case 2: return launch_gen_p<T, 2, STAR>(cfg, al, state, n, iters, out, s);
    default: return launch_gen_p<T, 4, STAR>(cfg, al, state, n, iters, out, s);
    }
}

} // namespace

bool launch_cfg_valid(const rngx_launch &cfg)
{
    return cfg.block >= 64 && cfg.block <= 1024 && cfg.block % 64 == 0 &&
           (cfg.chunks == 1 || cfg.chunks == 2 || cfg.chunks == 4) && cfg.nontemporal <= 1 &&
           (cfg.pace_gbs == 0 || (cfg.pace_gbs >= 1000 && cfg.pace_gbs <= 20000));
}

hipError_t launch_init(uint64_t *state, uint32_t n, const SeedMix &mix, hipStream_t s)
{
    const uint32_t block = 256;
    uint64_t blocks = ((uint64_t)n + block - 1) / block;
    if (blocks > 65536)
        blocks = 65536;
    init_kernel<<<dim3((uint32_t)blocks), dim3(block), 0, s>>>(state, n, mix);
    return hipGetLastError();
}

hipError_t launch_gen(const rngx_launch &cfg, bool u32, bool star, uint64_t *state, uint32_t n,
                      uint32_t iters, void *out, hipStream_t s)
{
    uint32_t *o32 = static_cast<uint32_t *>(out);
    uint64_t *o64 = static_cast<uint64_t *>(out);
    if (u32)
        return star ? launch_gen_typed<uint32_t, true>(cfg, state, n, iters, o32, s)
                    : launch_gen_typed<uint32_t, false>(cfg, state, n, iters, o32, s);
    return star ? launch_gen_typed<uint64_t, true>(cfg, state, n, iters, o64, s)
                : launch_gen_typed<uint64_t, false>(cfg, state, n, iters, o64, s);
}

} // namespace rngx
