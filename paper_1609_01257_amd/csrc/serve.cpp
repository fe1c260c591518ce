// Serving: a request loop over resident generator states.
//
// rngx_serve_start seeds n_states base states once (the init kernel) and
// keeps them on the device. A request names one stream g and a length L; at
// submission it reserves the next L values of g (its cursor c advances by
// L), so its result, V(seed, g, c + t) for t < L, is fixed when it is
// submitted and does not depend on which requests it is later batched with
// or when it runs.
//
// One scheduler thread moves requests through three stages:
//   pending  -> admitted: FIFO, as soon as the output pool (a caller-owned
//               device buffer) has room for L * 8 bytes;
//   admitted -> in flight: whenever one of the K launch streams is idle,
//               every admitted request (up to max_batch) goes into one
//               launch of the batched kernel, whose table the request's
//               stream start is jumped to from its resident base state;
//   in flight -> done: the stream's completion event is polled; latency is
//               measured from submission to the moment completion is seen.
// So requests arriving while others run are admitted and launched on another
// stream as soon as memory and a stream free up (continuous batching), and
// up to K batches overlap on the device. A consumer reads a done request's
// values in the pool and releases them; requests submitted with
// RNGX_SERVE_AUTORELEASE free their memory on completion.
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.h"
#include "pool.h"

namespace rngx {
namespace {

using Clock = std::chrono::steady_clock;

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               Clock::now().time_since_epoch())
        .count();
}

enum : uint8_t { ST_PENDING, ST_ADMITTED, ST_INFLIGHT, ST_DONE };

struct SReq {
    uint32_t gid;
    uint8_t state;
    bool autorelease;
    uint64_t offset, length;
    uint64_t t_arrive, t_admit, t_launch, t_done;
    uint64_t pool_off, pool_seq;
    bool live;
};

// A launch slot (staging buffers + completion event). Slots are spread over
// the launch streams, SLOTS_PER_STREAM each, so every stream can hold a
// batch queued behind the one it runs: batches that run side by side and
// finish together do not leave the device idle while the host refills.
constexpr uint32_t SLOTS_PER_STREAM = 2;

struct Flight {
    BatchSlot slot;
    hipStream_t stream = nullptr;
    uint32_t stream_index = 0;
    std::vector<uint64_t> tickets;
    bool busy = false;
};

struct Server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool active = false, stopping = false;
    int device = -1;
    uint64_t seed = 0;
    uint32_t n_states = 0;
    uint64_t *d_states = nullptr;
    char *pool = nullptr;
    uint64_t pool_bytes = 0;
    PoolRing alloc;
    std::vector<uint64_t> cursor;
    TicketTable<SReq> reqs;
    std::deque<uint64_t> pending;
    std::deque<uint64_t> admitted;
    std::vector<Flight> flights;
    std::vector<hipStream_t> streams;
    uint32_t max_batch = 1024;
    uint64_t max_pending = 1u << 20;
    uint32_t max_inflight = 2;
    bool star = false; // the output scrambler, fixed at start
    rngx_batch_cfg cfg{256, 4, 0, 0, 16, 1, 0, 0, 0, 0};
    std::thread worker;
    int worker_rc = RNGX_OK;
    std::string worker_msg;
    std::atomic<uint64_t> submit_seq{0}; // bumped by every submission (lock-free peek)
    // statistics
    std::vector<uint64_t> lat_ns, wait_ns, launch_ns, exec_ns, lag_ns;
    uint64_t submitted = 0, completed = 0, released = 0, batches = 0, batch_reqs = 0;
    uint64_t bytes_done = 0, t_first = 0, t_last = 0, max_pending_seen = 0, stalls = 0;
    bool stalled = false;
};

Server &SV()
{
    static Server *s = new Server;
    return *s;
}

void complete_flight(Server &s, Flight &f)
{
    const uint64_t t = now_ns();
    for (uint64_t tk : f.tickets) {
        SReq *rp = s.reqs.find(tk);
        if (!rp)
            continue;
        SReq &r = *rp;
        r.t_done = t;
        s.lat_ns.push_back(t - r.t_arrive);
        s.launch_ns.push_back(r.t_launch - r.t_arrive);
        s.exec_ns.push_back(t - r.t_launch);
        s.bytes_done += r.length * 8;
        ++s.completed;
        s.t_last = t;
        if (r.autorelease) {
            s.alloc.release(r.pool_seq);
            ++s.released;
            s.reqs.erase(tk);
        } else {
            r.state = ST_DONE;
        }
    }
    f.tickets.clear();
    f.busy = false;
}

// Admit, FIFO, while the pool has room for the request at the head.
bool admit(Server &s)
{
    bool progress = false;
    while (!s.pending.empty()) {
        SReq &r = *s.reqs.find(s.pending.front());
        uint64_t off = 0, seq = 0;
        if (!s.alloc.alloc(r.length * 8, &off, &seq)) {
            if (!s.stalled) {
                ++s.stalls;
                s.stalled = true;
            }
            break;
        }
        s.stalled = false;
        r.pool_off = off;
        r.pool_seq = seq;
        r.state = ST_ADMITTED;
        r.t_admit = now_ns();
        s.wait_ns.push_back(r.t_admit - r.t_arrive);
        s.admitted.push_back(s.pending.front());
        s.pending.pop_front();
        progress = true;
    }
    return progress;
}

// Batches of at most this many (padded) values (64 MiB) are latency-bound:
// they run one wave per small item, and one may run above the in-flight
// cap. Batches of a few requests of up to 2^22 values each stay below it
// (Poisson runs at 2k/10k/50k req/s, p99 55/55/69 us against 65/60/76-84
// with 2^20; the backlog's multi-GB batches are unaffected).
constexpr uint64_t kSmallBatchValues = 1u << 23;

// Launch schedule of a served batch of `values` (padded) values. Small
// batches are latency-bound: one wave per 1,024-value item (S = 16) spreads
// a request over the most waves, each storing soonest (Poisson runs at
// 2k/10k/50k req/s: p50 23/23/28 us against 28/27/33 with 4,096-value
// items). Larger ones run in the grouped order (S = 16, groups of 32
// wavefronts, 8 steps per region, schedule 6,250 GB/s: the batch
// autotuner's pick on the 4,096-stream table), which served a 243 GB
// backlog at 5.85 TB/s (median of three) against 5.52 for the persistent
// grid with S = 256 and 3.18 with the schedule halved for two batches in
// flight; the persistent grid had measured 5.45-5.51 against 4.90-4.97
// for one wave per item.
void serve_schedule(uint64_t values, rngx_batch_cfg &cfg)
{
    const bool small = values <= kSmallBatchValues;
    cfg.values_per_lane = 16;
    cfg.waves_per_block = 4;
    cfg.row_values = 16;
    cfg.per_item = small ? 1u : 0u;
    cfg.run_items = small ? 1u : 0u;
    cfg.group = small ? 0u : 32u;
    cfg.group_steps = small ? 0u : 8u;
    cfg.pace_gbs = small ? 0u : 6250u;
}

// Whether the next batch (the first max_batch admitted requests, padded as
// launch_admitted pads them) would be small.
bool next_batch_small(Server &s)
{
    uint64_t values = 0;
    uint32_t k = 0;
    for (uint64_t tk : s.admitted) {
        if (k++ == s.max_batch)
            break;
        values += (s.reqs.find(tk)->length + 15) & ~(uint64_t)15;
        if (values > kSmallBatchValues)
            return false;
    }
    return true;
}

int launch_admitted(Server &s, Flight &f, std::vector<StageReq> &items, const SeedMix &mix)
{
    items.clear();
    uint64_t vbase = 0;
    while (!s.admitted.empty() && items.size() < s.max_batch) {
        const uint64_t tk = s.admitted.front();
        s.admitted.pop_front();
        SReq &r = *s.reqs.find(tk);
        StageReq q;
        q.offset = r.offset;
        q.length = r.length;
        q.vbase = vbase;
        q.dst = reinterpret_cast<uint64_t *>(s.pool + r.pool_off);
        q.gid = r.gid;
        q.mix = mix;
        items.push_back(q);
        // Next request starts on a 16-value (128-byte) boundary of the
        // virtual index space, so its lines are whole in its own slice.
        vbase += (r.length + 15) & ~(uint64_t)15;
        r.state = ST_INFLIGHT;
        f.tickets.push_back(tk);
    }
    rngx_batch_cfg cfg = s.cfg;
    serve_schedule(vbase, cfg);
    int rc = batch_stage_items(f.slot, items.data(), (uint32_t)items.size(), cfg.values_per_lane,
                               s.d_states);
    if (rc == RNGX_OK)
        rc = batch_launch(f.slot, cfg, s.star, f.stream, true, "SERVE_KERNEL");
    const uint64_t t = now_ns();
    for (uint64_t tk : f.tickets)
        s.reqs.find(tk)->t_launch = t;
    if (rc == RNGX_OK) {
        f.busy = true;
        ++s.batches;
        s.batch_reqs += items.size();
    } else {
        // The batch never ran: its requests must never be reported done.
        // The caller records the failure, which every waiter then receives.
        f.tickets.clear();
    }
    return rc;
}

// Spin for about `ns` nanoseconds without the lock.
void spin_for(uint64_t ns)
{
    const uint64_t until = now_ns() + ns;
    while (now_ns() < until)
        __builtin_ia32_pause();
}

void worker_main(Server *sp)
{
    Server &s = *sp;
    const hipError_t dev_e = hipSetDevice(s.device);
    // Timed waits of this thread should not be stretched by the default
    // 50 us timer slack.
    (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
    std::vector<StageReq> items;
    std::unique_lock<std::mutex> lk(s.mu);
    if (dev_e != hipSuccess) {
        // Nothing can be launched from this thread: every waiter gets this.
        s.worker_rc = hip_fail(dev_e, "serve: hipSetDevice (scheduler thread)");
        s.worker_msg = rngx_last_error();
    }
    const SeedMix mix = seed_mix(s.seed); // unused by the kernel: states are resident
    for (;;) {
        bool progress = false, busy = false;
        for (Flight &f : s.flights) {
            if (!f.busy)
                continue;
            const hipError_t q = hipEventQuery(f.slot.done);
            if (q == hipSuccess) {
                complete_flight(s, f);
                progress = true;
            } else if (q != hipErrorNotReady) {
                s.worker_rc = hip_fail(q, "serve: batch completion");
                s.worker_msg = rngx_last_error();
                f.tickets.clear();
                f.busy = false;
            } else {
                busy = true;
            }
        }
        // Once stopping, nothing new is admitted or launched; batches already
        // in flight still write into the pool, so they are waited for.
        if (!s.stopping)
            progress |= admit(s);
        // After a failure nothing more is launched; waiters get the error.
        while (!s.stopping && !s.worker_rc && !s.admitted.empty()) {
            uint32_t inflight = 0;
            for (const Flight &f : s.flights)
                inflight += f.busy;
            // The cap keeps throughput-bound batches from competing on the
            // device; a small, latency-bound batch may run one above it
            // rather than wait (at 50k req/s with a cap of 2 and no such
            // allowance, p50 latency measured 28-45 us).
            if (inflight >= s.max_inflight &&
                (inflight > s.max_inflight || !next_batch_small(s)))
                break;
            // An idle slot on the stream with the fewest batches in flight.
            Flight *idle = nullptr;
            uint32_t best = ~0u;
            for (Flight &f : s.flights) {
                if (f.busy)
                    continue;
                uint32_t load = 0;
                for (const Flight &o : s.flights)
                    load += o.busy && o.stream_index == f.stream_index;
                if (load < best) {
                    best = load;
                    idle = &f;
                }
            }
            if (!idle)
                break;
            const int rc = launch_admitted(s, *idle, items, mix);
            if (rc) {
                s.worker_rc = rc;
                s.worker_msg = rngx_last_error();
                break;
            }
            busy = progress = true;
        }
        if (progress)
            s.cv_done.notify_all();
        if (s.stopping && !busy)
            break;
        if (!progress) {
            if (busy) {
                // Batches in flight: poll their events again shortly.
                lk.unlock();
                spin_for(2000);
                lk.lock();
            } else {
                // Idle: watch for a submission for 1 ms (two gaps between
                // arrivals at 2,000 requests/s), then sleep: a request that
                // arrives while this thread sleeps waits for its wake-up.
                const uint64_t seq = s.submit_seq.load(std::memory_order_acquire);
                lk.unlock();
                const uint64_t until = now_ns() + 1000000;
                while (s.submit_seq.load(std::memory_order_acquire) == seq && now_ns() < until)
                    __builtin_ia32_pause();
                lk.lock();
                // Nothing can move until a submission or a release (both wake
                // this thread): no requests, or the pool is full of results
                // that their consumers still hold.
                if (s.submit_seq.load(std::memory_order_acquire) == seq && !s.stopping &&
                    (s.pending.empty() || s.stalled) && s.admitted.empty())
                    s.cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
        }
    }
}

void reset_stats_locked(Server &s)
{
    s.lat_ns.clear();
    s.wait_ns.clear();
    s.launch_ns.clear();
    s.exec_ns.clear();
    s.lag_ns.clear();
    s.submitted = s.completed = s.released = s.batches = s.batch_reqs = 0;
    s.bytes_done = s.t_first = s.t_last = s.max_pending_seen = s.stalls = 0;
    s.stalled = false;
    s.alloc.reset_peak(); // live allocations stay
}

double pct(std::vector<uint64_t> &v, double p)
{
    if (v.empty())
        return 0.0;
    const size_t k = (size_t)std::min<double>((double)v.size() - 1, p / 100.0 * (double)v.size());
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k] * 1e-3;
}

void fill_stats_locked(Server &s, rngx_serve_report *o)
{
    std::memset(o, 0, sizeof *o);
    o->submitted = s.submitted;
    o->completed = s.completed;
    o->released = s.released;
    o->pending = s.pending.size();
    o->admitted = s.admitted.size();
    for (const Flight &f : s.flights)
        o->inflight_batches += f.busy;
    o->batches = s.batches;
    o->bytes = s.bytes_done;
    o->elapsed_s = s.t_last > s.t_first ? (s.t_last - s.t_first) * 1e-9 : 0.0;
    o->gbs = o->elapsed_s > 0 ? s.bytes_done / o->elapsed_s / 1e9 : 0.0;
    std::vector<uint64_t> lat = s.lat_ns, wait = s.wait_ns;
    o->lat_p50_us = pct(lat, 50.0);
    o->lat_p99_us = pct(lat, 99.0);
    o->lat_max_us = lat.empty() ? 0.0 : *std::max_element(lat.begin(), lat.end()) * 1e-3;
    double sum = 0;
    for (uint64_t v : s.lat_ns)
        sum += (double)v;
    o->lat_mean_us = s.lat_ns.empty() ? 0.0 : sum / s.lat_ns.size() * 1e-3;
    o->wait_p50_us = pct(wait, 50.0);
    o->wait_p99_us = pct(wait, 99.0);
    std::vector<uint64_t> la = s.launch_ns, ex = s.exec_ns;
    o->launch_p50_us = pct(la, 50.0);
    o->launch_p99_us = pct(la, 99.0);
    o->exec_p50_us = pct(ex, 50.0);
    o->exec_p99_us = pct(ex, 99.0);
    o->max_pending = s.max_pending_seen;
    o->admission_stalls = s.stalls;
    o->mean_batch_requests = s.batches ? (double)s.batch_reqs / s.batches : 0.0;
    o->pool_bytes = s.pool_bytes;
    o->pool_used_bytes = s.alloc.used();
    o->pool_peak_bytes = s.alloc.peak();
    std::vector<uint64_t> lag = s.lag_ns;
    o->lag_p50_us = pct(lag, 50.0);
    o->lag_p99_us = pct(lag, 99.0);
    o->lag_max_us = lag.empty() ? 0.0 : *std::max_element(lag.begin(), lag.end()) * 1e-3;
}

int check_request_locked(Server &s, uint32_t stream_id, uint64_t length, uint32_t flags)
{
    if (!s.active || s.stopping)
        return set_error(RNGX_E_NOINIT, "serve: the server is not running");
    if (stream_id >= s.n_states)
        return set_error(RNGX_E_INVAL, "serve: stream %u out of range (%u streams)", stream_id,
                         s.n_states);
    if (length == 0 || length > s.pool_bytes / 8)
        return set_error(RNGX_E_INVAL, "serve: length %llu is 0 or larger than the pool",
                         (unsigned long long)length);
    if (flags & ~(uint32_t)RNGX_SERVE_AUTORELEASE)
        return set_error(RNGX_E_INVAL, "serve: unknown flags 0x%x", flags);
    if (s.cursor[stream_id] > UINT64_MAX - length)
        return set_error(RNGX_E_INVAL, "serve: stream %u would pass value number 2^64 - 1",
                         stream_id);
    if (s.worker_rc)
        return set_error(s.worker_rc, "serve: scheduler failed: %s", s.worker_msg.c_str());
    return RNGX_OK;
}

// Tell the scheduler that requests were queued (or memory freed).
void wake_worker(Server &s)
{
    s.submit_seq.fetch_add(1, std::memory_order_release);
    s.cv_work.notify_one();
}

// Wait (or fail with BUSY) until one more request may be pending.
int make_room_locked(Server &s, std::unique_lock<std::mutex> &lk, bool wait)
{
    while (s.pending.size() >= s.max_pending) {
        if (!wait)
            return set_error(RNGX_E_BUSY, "serve: %llu requests already pending",
                             (unsigned long long)s.pending.size());
        // The pending requests (some perhaps queued by this very caller) are
        // what must move for room to appear.
        wake_worker(s);
        s.cv_done.wait(lk);
        if (!s.active || s.stopping)
            return set_error(RNGX_E_NOINIT, "serve: the server stopped");
    }
    return RNGX_OK;
}

// t_sched: the request's scheduled arrival (0: now, i.e. its submission).
uint64_t enqueue_locked(Server &s, uint32_t stream_id, uint64_t length, uint32_t flags,
                        uint64_t t_sched = 0)
{
    SReq r;
    r.gid = stream_id;
    r.state = ST_PENDING;
    r.autorelease = (flags & RNGX_SERVE_AUTORELEASE) != 0;
    r.offset = s.cursor[stream_id];
    r.length = length;
    const uint64_t t_now = now_ns();
    r.t_arrive = t_now;
    if (t_sched) {
        // Latency counts from the scheduled arrival; the submitter's delay
        // is recorded on its own.
        r.t_arrive = std::min(t_sched, t_now);
        s.lag_ns.push_back(t_now - r.t_arrive);
    }
    r.t_admit = r.t_launch = r.t_done = 0;
    r.pool_off = r.pool_seq = 0;
    r.live = true;
    s.cursor[stream_id] += length;
    const uint64_t tk = s.reqs.next_ticket();
    s.reqs.add(r);
    s.pending.push_back(tk);
    ++s.submitted;
    if (!s.t_first)
        s.t_first = r.t_arrive;
    s.max_pending_seen = std::max<uint64_t>(s.max_pending_seen, s.pending.size());
    return tk;
}

int submit_impl(uint32_t stream_id, uint64_t length, uint32_t flags, uint64_t *ticket, bool wait)
{
    Server &s = SV();
    std::unique_lock<std::mutex> lk(s.mu);
    clear_error();
    if (!ticket)
        return set_error(RNGX_E_INVAL, "serve: ticket is NULL");
    int rc = check_request_locked(s, stream_id, length, flags);
    if (rc == RNGX_OK)
        rc = make_room_locked(s, lk, wait);
    if (rc)
        return rc;
    *ticket = enqueue_locked(s, stream_id, length, flags);
    wake_worker(s);
    return RNGX_OK;
}

// Submit k requests under one lock acquisition (tickets and scheduled
// arrival times optional).
int submit_many_impl(const uint32_t *ids, const uint64_t *lengths, uint64_t k, uint32_t flags,
                     uint64_t *tickets, const uint64_t *t_sched = nullptr)
{
    Server &s = SV();
    std::unique_lock<std::mutex> lk(s.mu);
    int rc = RNGX_OK;
    uint64_t i = 0;
    for (; i < k; ++i) {
        rc = check_request_locked(s, ids[i], lengths[i], flags);
        if (rc == RNGX_OK)
            rc = make_room_locked(s, lk, true);
        if (rc)
            break;
        const uint64_t tk = enqueue_locked(s, ids[i], lengths[i], flags,
                                           t_sched ? t_sched[i] : 0);
        if (tickets)
            tickets[i] = tk;
    }
    // The requests queued before a failure stand, so they are scheduled too.
    if (i > 0)
        wake_worker(s);
    return rc;
}

void stop_locked(Server &s, std::unique_lock<std::mutex> &lk)
{
    if (!s.active)
        return;
    s.stopping = true;
    s.cv_work.notify_all();
    s.cv_done.notify_all();
    if (s.worker.joinable()) {
        lk.unlock();
        s.worker.join();
        lk.lock();
    }
    for (Flight &f : s.flights)
        release_slot(f.slot);
    s.flights.clear();
    for (hipStream_t st : s.streams)
        if (st)
            RNGX_NOTE(hipStreamDestroy(st));
    s.streams.clear();
    if (s.d_states)
        RNGX_NOTE(hipFree(s.d_states));
    s.d_states = nullptr;
    s.reqs.clear(s.reqs.next_ticket()); // tickets stay unique across restarts
    s.pending.clear();
    s.admitted.clear();
    s.cursor.clear();
    s.cursor.shrink_to_fit();
    s.alloc.reset(0);
    s.active = s.stopping = false;
}

} // namespace

void release_server()
{
    Server &s = SV();
    std::unique_lock<std::mutex> lk(s.mu);
    stop_locked(s, lk);
}

} // namespace rngx

using namespace rngx;

extern "C" int rngx_serve_start(uint64_t seed, uint32_t n_states, void *pool, uint64_t pool_bytes,
                                uint32_t n_streams, uint32_t max_batch)
{
    Server &s = SV();
    std::unique_lock<std::mutex> lk(s.mu);
    clear_error();
    if (s.active)
        return set_error(RNGX_E_BUSY, "serve: already running; call rngx_serve_stop first");
    if (n_states == 0 || !pool || pool_bytes < 256 || n_streams == 0 || n_streams > 16 ||
        max_batch == 0)
        return set_error(RNGX_E_INVAL, "serve: need n_states >= 1, a pool of >= 256 bytes, "
                                       "1..16 streams and max_batch >= 1");
    if (reinterpret_cast<uintptr_t>(pool) & 255u)
        return set_error(RNGX_E_INVAL, "serve: pool must be 256-byte aligned");
    int dev = -1;
    RNGX_HIP(hipGetDevice(&dev));
    int rc = batch_tables_locked(nullptr, nullptr, nullptr);
    if (rc)
        return rc;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, (size_t)n_states * sizeof(uint64_t));
    if (e != hipSuccess)
        return hip_fail(e, "serve: hipMalloc (resident states)");
    s.d_states = static_cast<uint64_t *>(p);
    s.streams.assign(n_streams, nullptr);
    for (hipStream_t &st : s.streams) {
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) {
            rc = hip_fail(e, "serve: hipStreamCreate");
            break;
        }
    }
    s.flights.resize((size_t)n_streams * SLOTS_PER_STREAM);
    for (size_t i = 0; i < s.flights.size(); ++i) {
        s.flights[i].stream_index = (uint32_t)(i % n_streams);
        s.flights[i].stream = s.streams[i % n_streams];
    }
    if (rc == RNGX_OK) {
        // The resident base states: the init kernel, once.
        hipStream_t s0 = s.streams[0];
        const int tok = prof::begin("INIT_KERNEL", s0);
        take_stray_error("before the serving init kernel launch");
        e = launch_init(s.d_states, n_states, seed_mix(seed), s0);
        prof::end(tok, s0);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s0);
        if (e != hipSuccess)
            rc = hip_fail(e, "serve: init kernel");
    }
    if (rc) {
        for (hipStream_t st : s.streams)
            if (st)
                RNGX_NOTE(hipStreamDestroy(st));
        s.streams.clear();
        s.flights.clear();
        RNGX_NOTE(hipFree(s.d_states));
        s.d_states = nullptr;
        return rc;
    }
    s.device = dev;
    s.seed = seed;
    s.n_states = n_states;
    s.pool = static_cast<char *>(pool);
    s.pool_bytes = pool_bytes;
    s.alloc.reset(pool_bytes & ~(uint64_t)255);
    s.cursor.assign(n_states, 0);
    s.max_batch = max_batch;
    // Batch sizes vary: launch directly (no graph) with a grid fitted to the
    // items, 4 waves per block, 8 waves per CU at most; S and the schedule
    // are chosen per batch.
    s.cfg = rngx_batch_cfg{256, 4, 0, 0, 16, 1, 0, 0, 0, 0};
    s.star = current_scrambler() == RNGX_SCRAMBLE_STAR;
    s.worker_rc = RNGX_OK;
    s.worker_msg.clear();
    reset_stats_locked(s);
    s.active = true;
    s.stopping = false;
    s.worker = std::thread(worker_main, &s);
    return RNGX_OK;
}

extern "C" int rngx_serve_submit(uint32_t stream_id, uint64_t length, uint32_t flags,
                                 uint64_t *ticket)
{
    return submit_impl(stream_id, length, flags, ticket, true);
}

extern "C" int rngx_serve_try_submit(uint32_t stream_id, uint64_t length, uint32_t flags,
                                     uint64_t *ticket)
{
    return submit_impl(stream_id, length, flags, ticket, false);
}

extern "C" int rngx_serve_submit_many(const uint32_t *stream_ids, const uint64_t *lengths,
                                      uint64_t k, uint32_t flags, uint64_t *tickets)
{
    clear_error();
    if (k && (!stream_ids || !lengths))
        return set_error(RNGX_E_INVAL, "serve: NULL request arrays");
    return submit_many_impl(stream_ids, lengths, k, flags, tickets);
}

extern "C" int rngx_serve_poll(uint64_t ticket, uint64_t **values, int *done)
{
    Server &s = SV();
    std::lock_guard<std::mutex> lk(s.mu);
    clear_error();
    if (!s.active)
        return set_error(RNGX_E_NOINIT, "serve: the server is not running");
    const SReq *rp = s.reqs.find(ticket);
    if (!rp)
        return set_error(RNGX_E_INVAL, "serve: unknown or released ticket %llu",
                         (unsigned long long)ticket);
    const SReq &r = *rp;
    if (done)
        *done = r.state == ST_DONE;
    if (values)
        *values = r.state == ST_PENDING ? nullptr
                                        : reinterpret_cast<uint64_t *>(s.pool + r.pool_off);
    return RNGX_OK;
}

extern "C" int rngx_serve_wait(uint64_t ticket, double timeout_s, uint64_t **values)
{
    Server &s = SV();
    std::unique_lock<std::mutex> lk(s.mu);
    clear_error();
    const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                             std::chrono::duration<double>(timeout_s));
    for (;;) {
        if (!s.active)
            return set_error(RNGX_E_NOINIT, "serve: the server is not running");
        const SReq *rp = s.reqs.find(ticket);
        if (!rp)
            return set_error(RNGX_E_INVAL, "serve: unknown or released ticket %llu",
                             (unsigned long long)ticket);
        if (rp->state == ST_DONE) {
            if (values)
                *values = reinterpret_cast<uint64_t *>(s.pool + rp->pool_off);
            return RNGX_OK;
        }
        if (s.worker_rc)
            return set_error(s.worker_rc, "serve: scheduler failed: %s", s.worker_msg.c_str());
        if (s.cv_done.wait_until(lk, deadline) == std::cv_status::timeout)
            return set_error(RNGX_E_BUSY, "serve: ticket %llu not done within %.3f s",
                             (unsigned long long)ticket, timeout_s);
    }
}

extern "C" int rngx_serve_release(uint64_t ticket)
{
    Server &s = SV();
    std::lock_guard<std::mutex> lk(s.mu);
    clear_error();
    if (!s.active)
        return set_error(RNGX_E_NOINIT, "serve: the server is not running");
    SReq *rp = s.reqs.find(ticket);
    if (!rp)
        return set_error(RNGX_E_INVAL, "serve: unknown or released ticket %llu",
                         (unsigned long long)ticket);
    if (rp->state != ST_DONE)
        return set_error(RNGX_E_BUSY, "serve: ticket %llu is not done yet",
                         (unsigned long long)ticket);
    s.alloc.release(rp->pool_seq);
    ++s.released;
    s.reqs.erase(ticket);
    wake_worker(s); // memory freed: admission may proceed
    return RNGX_OK;
}

extern "C" int rngx_serve_stats(rngx_serve_report *out)
{
    Server &s = SV();
    std::lock_guard<std::mutex> lk(s.mu);
    clear_error();
    if (!out)
        return set_error(RNGX_E_INVAL, "serve: stats is NULL");
    if (!s.active)
        return set_error(RNGX_E_NOINIT, "serve: the server is not running");
    fill_stats_locked(s, out);
    return RNGX_OK;
}

extern "C" int rngx_serve_reset_stats(void)
{
    Server &s = SV();
    std::lock_guard<std::mutex> lk(s.mu);
    clear_error();
    if (!s.active)
        return set_error(RNGX_E_NOINIT, "serve: the server is not running");
    reset_stats_locked(s);
    return RNGX_OK;
}

extern "C" int rngx_serve_run_trace(const double *arrival_s, const uint32_t *stream_id,
                                    const uint64_t *length, uint64_t k, double timeout_s,
                                    rngx_serve_report *out)
{
    clear_error();
    if (k && (!arrival_s || !stream_id || !length))
        return set_error(RNGX_E_INVAL, "serve: NULL trace arrays");
    {
        Server &s = SV();
        std::lock_guard<std::mutex> lk(s.mu);
        if (!s.active)
            return set_error(RNGX_E_NOINIT, "serve: the server is not running");
        reset_stats_locked(s);
    }
    // Scheduled arrival of every request, on the clock the server stamps with.
    std::vector<uint64_t> sched(k);
    const uint64_t t0 = now_ns();
    for (uint64_t i = 0; i < k; ++i)
        sched[i] = t0 + (uint64_t)(arrival_s[i] * 1e9);
    uint64_t i = 0;
    while (i < k) {
        const uint64_t due = sched[i];
        uint64_t t = now_ns();
        while (t < due) {
            __builtin_ia32_pause();
            t = now_ns();
        }
        // Every request whose arrival time has passed is submitted now, in
        // chunks of at most 512 so that the scheduler can start launching
        // while a large backlog is still being submitted.
        uint64_t j = i + 1;
        while (j < k && j - i < 512 && sched[j] <= t)
            ++j;
        const int rc = submit_many_impl(stream_id + i, length + i, j - i, RNGX_SERVE_AUTORELEASE,
                                        nullptr, sched.data() + i);
        if (rc)
            return rc;
        i = j;
    }
    Server &s = SV();
    std::unique_lock<std::mutex> lk(s.mu);
    const auto deadline = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                             std::chrono::duration<double>(timeout_s));
    while (s.completed < s.submitted) {
        if (s.worker_rc)
            return set_error(s.worker_rc, "serve: scheduler failed: %s", s.worker_msg.c_str());
        if (s.cv_done.wait_until(lk, deadline) == std::cv_status::timeout)
            return set_error(RNGX_E_BUSY, "serve: trace not drained within %.1f s", timeout_s);
    }
    if (out)
        fill_stats_locked(s, out);
    return RNGX_OK;
}

extern "C" int rngx_serve_set_max_pending(uint64_t max_pending)
{
    Server &s = SV();
    std::lock_guard<std::mutex> lk(s.mu);
    clear_error();
    if (max_pending == 0)
        return set_error(RNGX_E_INVAL, "serve: max_pending must be >= 1");
    s.max_pending = max_pending;
    s.cv_done.notify_all();
    return RNGX_OK;
}

extern "C" int rngx_serve_set_max_inflight(uint32_t max_inflight)
{
    Server &s = SV();
    std::lock_guard<std::mutex> lk(s.mu);
    clear_error();
    if (max_inflight == 0 || max_inflight > 32)
        return set_error(RNGX_E_INVAL, "serve: max_inflight must be in 1..32");
    s.max_inflight = max_inflight;
    s.cv_work.notify_all();
    return RNGX_OK;
}

extern "C" int rngx_serve_stop(void)
{
    Server &s = SV();
    std::unique_lock<std::mutex> lk(s.mu);
    clear_error();
    stop_locked(s, lk);
    return RNGX_OK;
}
