// Device-to-host copy kernel for the streaming pipeline.
//
// The paper's READ_BUFFER step is a device-to-host transfer of one output
// buffer (Section 5). A runtime copy (hipMemcpyAsync) that must wait for a
// kernel on another stream ran at well under half of the host link's rate
// on MI355X, while a kernel waiting for a kernel does not pay that cost. So
// the pipeline copies with this kernel: it reads the device buffer and
// stores straight into page-locked host memory mapped into the GPU's address
// space, 16 bytes per lane with non-temporal stores, grid-stride. PCIe write
// bandwidth, not HBM, bounds it; a few hundred waves keep enough writes in
// flight.
#include "internal.h"

namespace rngx {
namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename V>
__global__ __launch_bounds__(256) void d2h_kernel(const V *__restrict__ src, V *__restrict__ dst,
                                                  uint64_t count)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // Four independent loads in flight per lane before their stores.
    for (; i + 3 * stride < count; i += 4 * stride) {
        V a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < count; i += stride)
        __builtin_nontemporal_store(src[i], dst + i);
}

} // namespace

hipError_t launch_d2h(const void *src, void *dst_mapped, size_t bytes, uint32_t blocks,
                      hipStream_t s)
{
    if (bytes == 0)
        return hipSuccess;
    const uintptr_t a = reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst_mapped);
    if ((a & 15u) == 0 && bytes % 16 == 0) {
        const uint64_t count = bytes / 16;
        const uint64_t need = (count + 255) / 256;
        d2h_kernel<u32x4><<<dim3((uint32_t)(need < blocks ? need : blocks)), dim3(256), 0, s>>>(
            static_cast<const u32x4 *>(src), static_cast<u32x4 *>(dst_mapped), count);
    } else {
        // Pipeline steps are whole 4-byte values; any other alignment is
        // copied one dword per lane.
        const uint64_t count = bytes / 4;
        const uint64_t need = (count + 255) / 256;
        d2h_kernel<uint32_t><<<dim3((uint32_t)(need < blocks ? need : blocks)), dim3(256), 0, s>>>(
            static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst_mapped), count);
    }
    return hipGetLastError();
}

} // namespace rngx
