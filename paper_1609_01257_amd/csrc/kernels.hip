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

// P chunk columns per lane; NT: non-temporal stores; ALIGNED: every row
// start is 16-byte aligned (out 16-byte aligned and n*sizeof(T) % 16 == 0).
template <typename T, int P, bool NT, bool ALIGNED, bool STAR>
__global__ __launch_bounds__(1024) void gen_kernel(uint64_t *__restrict__ state, uint32_t n,
                                                   uint32_t iters, T *__restrict__ out)
{
    typedef Vec16<T> VT;
    constexpr int E = VT::E;
    constexpr uint64_t WAVE_ITEMS = 64ull * P * E;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t wbase = wave * WAVE_ITEMS;
    if (wbase >= n)
        return;

    uint64_t x[P][E];
    if (wbase + WAVE_ITEMS <= n) {
        // Fast path: every chunk of this wave is complete.
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const uint64_t g = wbase + (uint64_t)p * 64 * E + (uint64_t)lane * E;
#pragma unroll
            for (int e = 0; e < E; ++e)
                x[p][e] = state[g + e];
        }
        for (uint32_t k = 0; k < iters; ++k) {
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
        return;
    }

    // Last, partial wave: element-wise guarded (the paper's gid < nseeds test).
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

template <typename T, int P, bool STAR>
hipError_t launch_gen_p(const rngx_launch &cfg, bool al, uint64_t *state, uint32_t n,
                        uint32_t iters, T *out, hipStream_t s)
{
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
           (cfg.chunks == 1 || cfg.chunks == 2 || cfg.chunks == 4) && cfg.nontemporal <= 1;
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
