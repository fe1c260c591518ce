// Two-stream, double-buffered device-to-host streaming of generator output
// (Section 5 and Fig. 2: kernels on one queue, device-to-host reads on
// another, device-side double buffering so that each kernel overlaps the
// previous read).
//
// Step k generates `iters_per_step` iterations into device buffer k % 2 on
// the generation stream and copies it into host slot k % host_slots on the
// copy stream. HIP events replace the paper's two semaphores:
//   - the copy of step k waits for the generator's own state_ready event,
//     recorded right after generation k;
//   - generation k waits for the end of the copy of step k - 2, which read
//     the same device buffer: the profiler's end event of that copy when it
//     was profiled, else `copy_done[k % 2]`.
// Here the output buffers are double-buffered, not the state (the state
// stays in a library buffer and, inside one launch, in registers), so
// generation of step k + 1 may run while step k is still being copied.
// If a consumer is given, it is called on this thread for every step in
// order once its copy is complete, and a host slot is reused only after the
// consumer has returned for the step it held (host-side multi-buffering, the
// paper's suggested improvement in Section 5).
#include <algorithm>
#include <vector>

#include "internal.h"

namespace rngx {

void release_pipeline_locked(Generator &g)
{
    if (g.pipe_copy)
        RNGX_NOTE(hipStreamSynchronize(g.pipe_copy));
    if (g.pipe_gen)
        RNGX_NOTE(hipStreamSynchronize(g.pipe_gen));
    for (int i = 0; i < 2; ++i) {
        if (g.copy_done[i])
            RNGX_NOTE(hipEventDestroy(g.copy_done[i]));
        g.copy_done[i] = nullptr;
    }
    if (g.pipe_gen)
        RNGX_NOTE(hipStreamDestroy(g.pipe_gen));
    if (g.pipe_copy)
        RNGX_NOTE(hipStreamDestroy(g.pipe_copy));
    g.pipe_gen = g.pipe_copy = nullptr;
}

namespace {

// A stream on a hardware queue of its own. HIP maps streams onto a small
// pool of hardware queues (four per process by default); once the pool is
// full, a new stream shares the least-used queue, and two streams on one
// queue run their work in submission order. The pipeline's two streams,
// created after the library's and the caller's other streams, could then
// share a queue, and the kernel of step k + 1 would wait behind the copy of
// step k: no overlap at all. A stream created with a compute-unit mask
// always gets a queue of its own; the mask here enables every compute unit.
// (Such a stream synchronises with the null stream like a default stream.)
int create_own_queue_stream(hipStream_t *s)
{
    int dev = -1, cus = 0;
    RNGX_HIP(hipGetDevice(&dev));
    RNGX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    uint32_t mask[32];
    const uint32_t words = (uint32_t)std::min(32, std::max(1, (cus + 31) / 32));
    for (uint32_t i = 0; i < words; ++i)
        mask[i] = 0xffffffffu;
    RNGX_HIP(hipExtStreamCreateWithCUMask(s, words, mask));
    return RNGX_OK;
}

int ensure_pipeline_locked(Generator &g)
{
    if (!g.pipe_gen) {
        int rc = create_own_queue_stream(&g.pipe_gen);
        if (rc)
            return rc;
    }
    if (!g.pipe_copy) {
        int rc = create_own_queue_stream(&g.pipe_copy);
        if (rc)
            return rc;
    }
    for (int i = 0; i < 2; ++i) {
        if (!g.copy_done[i])
            RNGX_HIP(hipEventCreateWithFlags(&g.copy_done[i], hipEventDisableTiming));
    }
    return RNGX_OK;
}

struct SlotEvents {
    std::vector<hipEvent_t> ev;
    ~SlotEvents()
    {
        for (hipEvent_t e : ev)
            RNGX_NOTE(hipEventDestroy(e));
    }
};

} // namespace
} // namespace rngx

using namespace rngx;

extern "C" int rngx_set_copy_mode(int mode, uint32_t blocks)
{
    Generator &g = generator();
    std::lock_guard<std::recursive_mutex> lk(g.mu);
    clear_error();
    if ((mode != RNGX_COPY_KERNEL && mode != RNGX_COPY_RUNTIME) || blocks == 0 || blocks > 65536)
        return set_error(RNGX_E_INVAL, "rngx_set_copy_mode: mode must be RNGX_COPY_KERNEL or "
                                       "RNGX_COPY_RUNTIME and blocks 1..65536");
    g.copy_mode = mode;
    g.copy_blocks = blocks;
    return RNGX_OK;
}

extern "C" int rngx_get_copy_mode(int *mode, uint32_t *blocks)
{
    Generator &g = generator();
    std::lock_guard<std::recursive_mutex> lk(g.mu);
    clear_error();
    if (mode)
        *mode = g.copy_mode;
    if (blocks)
        *blocks = g.copy_blocks;
    return RNGX_OK;
}

extern "C" int rngx_inject_copy_failure(uint64_t step)
{
    Generator &g = generator();
    std::lock_guard<std::recursive_mutex> lk(g.mu);
    clear_error();
    g.fail_copy_at = step;
    return RNGX_OK;
}

extern "C" int rngx_stream_to_host(uint32_t n_steps, uint32_t iters_per_step, int u32,
                                   void *dev0, void *dev1, size_t dev_bytes, void *host,
                                   uint32_t host_slots, rngx_consume_fn consume, void *user,
                                   void *gen_stream, void *copy_stream)
{
    Generator &g = generator();
    std::lock_guard<std::recursive_mutex> lk(g.mu);
    clear_error();
    if (!g.inited)
        return set_error(RNGX_E_NOINIT, "rngx_stream_to_host called before rngx_init");
    if (n_steps == 0)
        return RNGX_OK;
    const size_t esize = u32 ? 4 : 8;
    if (iters_per_step == 0)
        return set_error(RNGX_E_INVAL, "stream_to_host: iters_per_step must be >= 1");
    if (!dev0 || !dev1 || dev0 == dev1)
        return set_error(RNGX_E_INVAL, "stream_to_host: need two distinct device buffers");
    if (reinterpret_cast<uintptr_t>(dev0) % esize || reinterpret_cast<uintptr_t>(dev1) % esize)
        return set_error(RNGX_E_INVAL, "stream_to_host: device buffers not %zu-byte aligned",
                         esize);
    if (!host || host_slots == 0)
        return set_error(RNGX_E_INVAL, "stream_to_host: need a host buffer with >= 1 slot");
    const unsigned __int128 step_bytes128 = (unsigned __int128)iters_per_step * g.n * esize;
    if (step_bytes128 > dev_bytes)
        return set_error(RNGX_E_INVAL,
                         "stream_to_host: a step needs %llu bytes but device buffers hold %zu",
                         (unsigned long long)step_bytes128, dev_bytes);
    const size_t step_bytes = (size_t)step_bytes128;
    if ((unsigned __int128)step_bytes * host_slots > (unsigned __int128)SIZE_MAX)
        return set_error(RNGX_E_INVAL, "stream_to_host: host buffer size overflows size_t");
    // The test hook applies to this call only.
    const uint64_t fail_at = g.fail_copy_at;
    g.fail_copy_at = UINT64_MAX;
    int rc = check_device_locked(g);
    if (rc)
        return rc;
    rc = ensure_pipeline_locked(g);
    if (rc)
        return rc;
    hipStream_t gs = gen_stream ? static_cast<hipStream_t>(gen_stream) : g.pipe_gen;
    hipStream_t cs = copy_stream ? static_cast<hipStream_t>(copy_stream) : g.pipe_copy;
    if (gs == cs)
        return set_error(RNGX_E_INVAL, "stream_to_host: generation and copy streams must differ");

    // Device-mapped address of the host buffer, for the copy kernel.
    char *hmapped = nullptr;
    if (g.copy_mode == RNGX_COPY_KERNEL) {
        void *p = nullptr;
        if (hipHostGetDevicePointer(&p, host, 0) == hipSuccess && p)
            hmapped = static_cast<char *>(p);
        else
            (void)hipGetLastError(); // its own error: not page-locked, so use the runtime copy
    }

    SlotEvents slots;
    if (consume) {
        slots.ev.resize(host_slots, nullptr);
        for (uint32_t i = 0; i < host_slots; ++i)
            RNGX_HIP(hipEventCreateWithFlags(&slots.ev[i], hipEventDisableTiming));
    }
    void *dev[2] = {dev0, dev1};
    hipEvent_t copy_dep[2] = {nullptr, nullptr}; // end of the copy that last read dev[b]
    char *hbase = static_cast<char *>(host);
    // On an error or an abort, wait for everything already enqueued on both
    // streams, so that no kernel or copy still uses the caller's buffers
    // when the call returns.
    auto drain = [&]() {
        RNGX_NOTE(hipStreamSynchronize(gs));
        RNGX_NOTE(hipStreamSynchronize(cs));
    };

    // A failed HIP call once work is queued: report it, after the drain.
    auto fail = [&](hipError_t e, const char *what) -> int {
        const int code = hip_fail(e, what);
        drain();
        return code;
    };
#define PIPE_HIP(call)                                   \
    do {                                                 \
        const hipError_t pipe_e_ = (call);               \
        if (pipe_e_ != hipSuccess)                       \
            return fail(pipe_e_, #call);                 \
    } while (0)

    auto consume_step = [&](uint64_t k) -> int {
        const uint32_t slot = (uint32_t)(k % host_slots);
        PIPE_HIP(hipEventSynchronize(slots.ev[slot]));
        if (consume(user, k, hbase + (size_t)slot * step_bytes, step_bytes) != 0)
            return set_error(RNGX_E_ABORTED, "stream_to_host: consumer stopped the stream at step "
                                             "%llu",
                             (unsigned long long)k);
        return RNGX_OK;
    };

    for (uint64_t k = 0; k < n_steps; ++k) {
        const uint32_t slot = (uint32_t)(k % host_slots);
        const int b = (int)(k & 1);
        if (consume && k >= host_slots) {
            rc = consume_step(k - host_slots);
            if (rc) {
                drain();
                return rc;
            }
        }
        if (k >= 2)
            PIPE_HIP(hipStreamWaitEvent(gs, copy_dep[b], 0));
        rc = generate_locked(g, iters_per_step, dev[b], gs, u32 != 0);
        if (rc) {
            drain();
            return rc;
        }
        // generate_locked recorded state_ready on gs right after the kernel:
        // it marks the generation's end, so no event of our own is queued.
        PIPE_HIP(hipStreamWaitEvent(cs, g.state_ready, 0));
        if (k == fail_at) {
            // Test hook: this step's copy "fails" before it is enqueued, as
            // a read error in the paper's communications thread would.
            const int code = set_error(RNGX_E_HIP,
                                       "stream_to_host: device-to-host copy of step %llu failed "
                                       "(forced by rngx_inject_copy_failure)",
                                       (unsigned long long)k);
            drain();
            return code;
        }
        const int tok = prof::begin("READ_BUFFER", cs);
        take_stray_error("before the device-to-host copy");
        hipError_t e = hmapped
                           ? launch_d2h(dev[b], hmapped + (size_t)slot * step_bytes, step_bytes,
                                        g.copy_blocks, cs)
                           : hipMemcpyAsync(hbase + (size_t)slot * step_bytes, dev[b], step_bytes,
                                            hipMemcpyDeviceToHost, cs);
        // The profiler's end event of the copy, when there is one, also
        // orders generation k + 2 after it (one marker fewer per step).
        hipEvent_t copied = prof::end_event(tok, cs);
        if (e != hipSuccess)
            return fail(e, hmapped ? "device-to-host copy kernel" : "hipMemcpyAsync (D2H)");
        if (!copied) {
            PIPE_HIP(hipEventRecord(g.copy_done[b], cs));
            copied = g.copy_done[b];
        }
        copy_dep[b] = copied;
        if (consume)
            PIPE_HIP(hipEventRecord(slots.ev[slot], cs));
    }
    if (consume) {
        const uint64_t first = n_steps > host_slots ? n_steps - host_slots : 0;
        for (uint64_t k = first; k < n_steps; ++k) {
            rc = consume_step(k);
            if (rc) {
                drain();
                return rc;
            }
        }
    }
    PIPE_HIP(hipStreamSynchronize(cs));
#undef PIPE_HIP
    return RNGX_OK;
}
