// C ABI of the generator: context, lifecycle, plain generation, errors.
//
// One process-wide context (Generator, internal.h) holds the library-owned
// state buffer, the library's own stream (for the init kernel) and the
// `state_ready` event that orders every use of the state across caller
// streams: a generate call makes its stream wait for `state_ready`,
// launches, and re-records it.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <vector>

#include <sys/syscall.h>
#include <unistd.h>

#include "internal.h"

namespace rngx {

static thread_local std::string t_last_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    // The error goes back to the caller through the return code: consume it,
    // so that an unrelated hipGetLastError (the library's before its next
    // launch, or the application's) does not report it a second time.
    (void)hipGetLastError();
    const int code = (e == hipErrorOutOfMemory) ? RNGX_E_NOMEM : RNGX_E_HIP;
    return set_error(code, "%s failed: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
}

void clear_error() { t_last_error.clear(); }

namespace {

// The notes of rngx_hip_notes: counts since the last clear and the most
// recent lines.
struct HipNotes {
    std::mutex mu;
    uint64_t released = 0, stray = 0;
    std::deque<std::string> last;
};
constexpr size_t kMaxNotes = 32;

HipNotes &hip_notes()
{
    static HipNotes *n = new HipNotes; // never destroyed: used until exit
    return *n;
}

void add_note(bool own, const char *what, hipError_t e)
{
    char buf[320];
    std::snprintf(buf, sizeof buf, "%s %s: %s (thread %ld)", own ? "released" : "stray", what,
                  hipGetErrorName(e), (long)syscall(SYS_gettid));
    HipNotes &n = hip_notes();
    std::lock_guard<std::mutex> lk(n.mu);
    ++(own ? n.released : n.stray);
    n.last.emplace_back(buf);
    if (n.last.size() > kMaxNotes)
        n.last.pop_front();
}

} // namespace

void note_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess)
        return;
    (void)hipGetLastError(); // this call's own error, recorded below
    add_note(true, what, e);
}

void take_stray_error(const char *where)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        add_note(false, where, e);
}

Generator &generator()
{
    static Generator *g = new Generator; // never destroyed: HIP may be gone at exit
    return *g;
}

namespace {

// Free the state of a previous init (waits for its last use first).
int release_state_locked(Generator &c)
{
    if (c.state_ready)
        RNGX_HIP(hipEventSynchronize(c.state_ready));
    if (c.state) {
        RNGX_HIP(hipFree(c.state));
        c.state = nullptr;
    }
    c.inited = false;
    c.n = 0;
    c.cursor = 0;
    return RNGX_OK;
}

// Free any previous state, make sure the library stream and event exist on
// the current device, allocate n states and open a new profiling window.
int fresh_state_locked(Generator &c, uint32_t n_states, const char *who)
{
    int rc = release_state_locked(c);
    if (rc)
        return rc;
    int dev = -1;
    RNGX_HIP(hipGetDevice(&dev));
    if (c.lib_stream && dev != c.device) {
        // Resources belong to another device: recreate them here (the
        // streaming pipeline's streams and events on first use).
        release_pipeline_locked(c);
        RNGX_NOTE(hipStreamDestroy(c.lib_stream));
        RNGX_NOTE(hipEventDestroy(c.state_ready));
        c.lib_stream = nullptr;
        c.state_ready = nullptr;
    }
    c.device = dev;
    if (!c.lib_stream)
        RNGX_HIP(hipStreamCreateWithFlags(&c.lib_stream, hipStreamNonBlocking));
    if (!c.state_ready)
        RNGX_HIP(hipEventCreateWithFlags(&c.state_ready, hipEventDisableTiming));
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)n_states * sizeof(uint64_t));
    if (e != hipSuccess) {
        (void)hipGetLastError(); // this allocation's own error, reported below
        return set_error(RNGX_E_NOMEM, "%s: cannot allocate %zu bytes of state: %s", who,
                         (size_t)n_states * sizeof(uint64_t), hipGetErrorString(e));
    }
    c.state = static_cast<uint64_t *>(p);
    return prof::start(c.lib_stream);
}

int generate_impl(uint32_t n_iters, void *out, void *stream, bool u32)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    return generate_locked(c, n_iters, out, static_cast<hipStream_t>(stream), u32);
}

} // namespace

int check_device_locked(const Generator &c)
{
    int dev = -1;
    RNGX_HIP(hipGetDevice(&dev));
    if (dev != c.device)
        return set_error(RNGX_E_INVAL,
                         "the generator lives on device %d but device %d is current", c.device,
                         dev);
    return RNGX_OK;
}

int generate_locked(Generator &c, uint32_t n_iters, void *out, hipStream_t s, bool u32)
{
    if (!c.inited)
        return set_error(RNGX_E_NOINIT, "generate called before rngx_init");
    if (n_iters == 0)
        return RNGX_OK;
    const size_t esize = u32 ? 4 : 8;
    if (!out)
        return set_error(RNGX_E_INVAL, "generate: out is NULL");
    if (reinterpret_cast<uintptr_t>(out) % esize)
        return set_error(RNGX_E_INVAL, "generate: out is not %zu-byte aligned", esize);
    const unsigned __int128 bytes = (unsigned __int128)n_iters * c.n * esize;
    if (bytes > (unsigned __int128)SIZE_MAX)
        return set_error(RNGX_E_INVAL, "generate: output size overflows size_t");
    if (c.cursor > UINT64_MAX - n_iters)
        return set_error(RNGX_E_INVAL, "generate: the cursor would pass value number 2^64 - 1");
    int rc = check_device_locked(c);
    if (rc)
        return rc;
    RNGX_HIP(hipStreamWaitEvent(s, c.state_ready, 0));
    const int tok = prof::begin("RNG_KERNEL", s);
    rngx_launch cfg = u32 ? c.cfg32 : c.cfg64;
    if (cfg.block == 0) {
        // The library's choice: the row-scheduled launch at 7,000 GB/s,
        // 6.8-7.1 TB/s at every size from 2^20 to 2^26 states x 256
        // iterations, u64 and u32, on MI355X (unscheduled: 5.4-6.5), with
        // a margin below the rates where a schedule falls behind.
        cfg = rngx_launch{512, 2, 1, 7000};
    }
    take_stray_error("before the rng kernel launch");
    hipError_t e = launch_gen(cfg, u32,
                              current_scrambler() == RNGX_SCRAMBLE_STAR, c.state, c.n, n_iters,
                              out, s);
    prof::end(tok, s);
    if (e != hipSuccess)
        return hip_fail(e, "rng kernel launch");
    RNGX_HIP(hipEventRecord(c.state_ready, s));
    c.cursor += n_iters;
    return RNGX_OK;
}

} // namespace rngx

using namespace rngx;

extern "C" {

int rngx_init(uint64_t seed, uint32_t n_states)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    if (n_states == 0)
        return set_error(RNGX_E_INVAL, "rngx_init: n_states must be at least 1");
    // Once per process: the tuning cache named by RNGX_TUNE_CACHE.
    static bool cache_applied = false;
    if (!cache_applied) {
        int rc = tune_cache_apply_env();
        if (rc)
            return rc;
        cache_applied = true;
    }
    int rc = fresh_state_locked(c, n_states, "rngx_init");
    if (rc)
        return rc;
    const int tok = prof::begin("INIT_KERNEL", c.lib_stream);
    take_stray_error("before the init kernel launch");
    hipError_t e = launch_init(c.state, n_states, seed_mix(seed), c.lib_stream);
    prof::end(tok, c.lib_stream);
    if (e != hipSuccess)
        return hip_fail(e, "init kernel launch");
    RNGX_HIP(hipEventRecord(c.state_ready, c.lib_stream));
    c.seed = seed;
    c.n = n_states;
    c.cursor = 0;
    c.inited = true;
    return RNGX_OK;
}

int rngx_get_state(uint64_t *states, uint32_t n, uint64_t *seed, uint64_t *cursor)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    if (!c.inited)
        return set_error(RNGX_E_NOINIT, "rngx_get_state called before rngx_init");
    if (!states || n != c.n)
        return set_error(RNGX_E_INVAL, "rngx_get_state: need a host array of %u states", c.n);
    int rc = check_device_locked(c);
    if (rc)
        return rc;
    RNGX_HIP(hipStreamWaitEvent(c.lib_stream, c.state_ready, 0));
    RNGX_HIP(hipMemcpyAsync(states, c.state, (size_t)n * sizeof(uint64_t),
                            hipMemcpyDeviceToHost, c.lib_stream));
    RNGX_HIP(hipStreamSynchronize(c.lib_stream));
    if (seed)
        *seed = c.seed;
    if (cursor)
        *cursor = c.cursor;
    return RNGX_OK;
}

int rngx_set_state(uint64_t seed, const uint64_t *states, uint32_t n, uint64_t cursor)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    if (!states || n == 0)
        return set_error(RNGX_E_INVAL, "rngx_set_state: need at least one state");
    for (uint32_t g = 0; g < n; ++g)
        if (states[g] == 0)
            return set_error(RNGX_E_INVAL, "rngx_set_state: state %u is 0", g);
    int rc = fresh_state_locked(c, n, "rngx_set_state");
    if (rc)
        return rc;
    RNGX_HIP(hipMemcpyAsync(c.state, states, (size_t)n * sizeof(uint64_t),
                            hipMemcpyHostToDevice, c.lib_stream));
    RNGX_HIP(hipStreamSynchronize(c.lib_stream));
    RNGX_HIP(hipEventRecord(c.state_ready, c.lib_stream));
    c.seed = seed;
    c.n = n;
    c.cursor = cursor;
    c.inited = true;
    return RNGX_OK;
}

int rngx_generate(uint32_t n_iters, uint64_t *out, void *stream)
{
    return generate_impl(n_iters, out, stream, false);
}

int rngx_generate_u32(uint32_t n_iters, uint32_t *out, void *stream)
{
    return generate_impl(n_iters, out, stream, true);
}

int rngx_info(uint64_t *seed, uint32_t *n_states, uint64_t *cursor)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    if (!c.inited)
        return set_error(RNGX_E_NOINIT, "rngx_info called before rngx_init");
    if (seed)
        *seed = c.seed;
    if (n_states)
        *n_states = c.n;
    if (cursor)
        *cursor = c.cursor;
    return RNGX_OK;
}

int rngx_shutdown(void)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    int rc = release_state_locked(c);
    release_pipeline_locked(c);
    release_server();
    release_batch();
    prof::release_all();
    if (c.state_ready)
        RNGX_NOTE(hipEventDestroy(c.state_ready));
    if (c.lib_stream)
        RNGX_NOTE(hipStreamDestroy(c.lib_stream));
    c.state_ready = nullptr;
    c.lib_stream = nullptr;
    c.device = -1;
    return rc;
}

const char *rngx_last_error(void) { return t_last_error.c_str(); }

int rngx_hip_notes(uint64_t *released, uint64_t *stray, char *text, size_t cap, int clear)
{
    clear_error();
    if (text && cap == 0)
        return set_error(RNGX_E_INVAL, "rngx_hip_notes: text given with cap 0");
    HipNotes &n = hip_notes();
    std::lock_guard<std::mutex> lk(n.mu);
    if (released)
        *released = n.released;
    if (stray)
        *stray = n.stray;
    if (text) {
        std::string all;
        for (const std::string &l : n.last)
            all += l + "\n";
        const size_t k = std::min(all.size(), cap - 1);
        std::memcpy(text, all.data(), k);
        text[k] = 0;
    }
    if (clear) {
        n.released = n.stray = 0;
        n.last.clear();
    }
    return RNGX_OK;
}

const char *rngx_strerror(int code)
{
    switch (code) {
    case RNGX_OK: return "RNGX_OK: success";
    case RNGX_E_INVAL: return "RNGX_E_INVAL: invalid argument";
    case RNGX_E_NOINIT: return "RNGX_E_NOINIT: generator not initialised";
    case RNGX_E_HIP: return "RNGX_E_HIP: HIP runtime error";
    case RNGX_E_NOMEM: return "RNGX_E_NOMEM: out of device memory";
    case RNGX_E_BUSY: return "RNGX_E_BUSY: resource full, retry later";
    case RNGX_E_ABORTED: return "RNGX_E_ABORTED: stopped by the caller's consumer";
    default: return "unknown rngx status code";
    }
}

int rngx_set_launch(int u32, const rngx_launch *cfg)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    if (!cfg || (cfg->block != 0 && !launch_cfg_valid(*cfg)))
        return set_error(RNGX_E_INVAL,
                         "rngx_set_launch: block must be 0 (automatic) or 64..1024 in steps of "
                         "64, chunks 1, 2 or 4, nontemporal 0 or 1, pace_gbs 0 or 1000..20000");
    (u32 ? c.cfg32 : c.cfg64) = *cfg;
    return RNGX_OK;
}

} // extern "C"

// The scrambler is read by the batched and served paths while they hold
// their own locks; an atomic keeps it out of every lock order.
static std::atomic<int> g_scrambler{RNGX_SCRAMBLE_NONE};

int rngx::current_scrambler() { return g_scrambler.load(std::memory_order_acquire); }

extern "C" {

int rngx_set_scrambler(int scrambler)
{
    clear_error();
    if (scrambler != RNGX_SCRAMBLE_NONE && scrambler != RNGX_SCRAMBLE_STAR)
        return set_error(RNGX_E_INVAL, "rngx_set_scrambler: unknown scrambler %d", scrambler);
    g_scrambler.store(scrambler, std::memory_order_release);
    return RNGX_OK;
}

int rngx_get_scrambler(int *scrambler)
{
    clear_error();
    if (!scrambler)
        return set_error(RNGX_E_INVAL, "rngx_get_scrambler: NULL");
    *scrambler = current_scrambler();
    return RNGX_OK;
}

int rngx_get_launch(int u32, rngx_launch *cfg)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    if (!cfg)
        return set_error(RNGX_E_INVAL, "rngx_get_launch: NULL");
    *cfg = u32 ? c.cfg32 : c.cfg64;
    return RNGX_OK;
}

int rngx_profile_start(void)
{
    Generator &c = generator();
    std::lock_guard<std::recursive_mutex> lk(c.mu);
    clear_error();
    if (!c.lib_stream)
        return set_error(RNGX_E_NOINIT, "rngx_profile_start called before rngx_init");
    return prof::start(c.lib_stream);
}

int rngx_profile_reset(void) { return rngx_profile_start(); }

int rngx_profile_stop(void)
{
    clear_error();
    return prof::stop();
}

int rngx_profile_enable(int on)
{
    clear_error();
    return prof::enable(on);
}

const char *rngx_profile(void)
{
    clear_error();
    return prof::summary();
}

int rngx_profile_stats(rngx_prof_stats *out)
{
    clear_error();
    if (!out)
        return set_error(RNGX_E_INVAL, "rngx_profile_stats: NULL");
    return prof::stats(out);
}

int rngx_profile_events(rngx_prof_event *out, uint32_t cap, uint32_t *n_out)
{
    clear_error();
    return prof::events(out, cap, n_out);
}

int rngx_profile_analyze(const rngx_prof_event *events, uint32_t n, double elapsed_s,
                         rngx_prof_stats *out)
{
    clear_error();
    return analyze_table(events, n, elapsed_s, out);
}

int rngx_profile_write(const rngx_prof_event *events, uint32_t n, const char *path, int format)
{
    clear_error();
    return write_table(events, n, path, format);
}

int rngx_profile_export(const char *path, int format)
{
    clear_error();
    uint32_t n = 0;
    int rc = prof::events(nullptr, 0, &n);
    if (rc)
        return rc;
    std::vector<rngx_prof_event> ev(n);
    uint32_t got = 0;
    rc = prof::events(ev.data(), n, &got);
    if (rc)
        return rc;
    ev.resize(std::min(n, got));
    return write_table(ev.data(), (uint32_t)ev.size(), path, format);
}

} // extern "C"
