// Event profiler: the semantics of the cf4ocl profiler module (Section 4.3)
// and of its summary (Fig. 3), on HIP events.
//
// Every timed operation records a start and an end HIP event on the stream
// it runs on. When the window is closed the events are resolved to
// nanoseconds relative to a reference event recorded when the window opened.
// The analysis aggregates durations per name, finds pairwise overlaps
// between operations on different streams with one sort and a sweep
// (O(E log E + E*Q) for Q streams, instead of examining every pair), and
// derives the effective time and the device/host split.
#include <algorithm>
#include <cerrno>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"

namespace rngx {

struct EventRow {
    uint32_t name; // index into the name table
    uint64_t queue;
    uint64_t start_ns;
    uint64_t end_ns;
};

// Analyse rows whose names are in `names`; fills `out`. Returns RNGX_OK or
// RNGX_E_INVAL (an event that ends before it starts).
static int analyze_rows(const std::vector<EventRow> &rows, const std::vector<std::string> &names,
                        double elapsed_s, rngx_prof_stats *out)
{
    std::memset(out, 0, sizeof(*out));
    const size_t nn = names.size();
    std::vector<uint64_t> sum(nn, 0), cnt(nn, 0);
    uint64_t total = 0;
    for (const EventRow &r : rows) {
        if (r.end_ns < r.start_ns)
            return set_error(RNGX_E_INVAL, "event '%s' ends before it starts",
                             names[r.name].c_str());
        sum[r.name] += r.end_ns - r.start_ns;
        cnt[r.name] += 1;
        total += r.end_ns - r.start_ns;
    }

    // Sweep in start order; `active` holds events that may still overlap a
    // later-starting one. An event a that started no later than e overlaps e
    // by min(a.end, e.end) - e.start when that is positive.
    std::vector<uint32_t> order(rows.size());
    for (uint32_t i = 0; i < order.size(); ++i)
        order[i] = i;
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (rows[a].start_ns != rows[b].start_ns)
            return rows[a].start_ns < rows[b].start_ns;
        return a < b;
    });
    std::map<std::pair<uint32_t, uint32_t>, uint64_t> pair_ns;
    std::vector<uint32_t> active;
    uint64_t overlap = 0;
    for (uint32_t idx : order) {
        const EventRow &e = rows[idx];
        size_t w = 0;
        for (size_t i = 0; i < active.size(); ++i) {
            const EventRow &a = rows[active[i]];
            if (a.end_ns <= e.start_ns)
                continue; // finished: cannot overlap e or anything after it
            active[w++] = active[i];
            if (a.queue == e.queue)
                continue;
            const uint64_t ov = std::min(a.end_ns, e.end_ns) - e.start_ns;
            if (ov == 0)
                continue;
            const uint32_t x = std::min(a.name, e.name), y = std::max(a.name, e.name);
            pair_ns[{x, y}] += ov;
            overlap += ov;
        }
        active.resize(w);
        active.push_back(idx);
    }

    out->n_events = rows.size();
    out->total_s = total * 1e-9;
    out->overlap_s = overlap * 1e-9;
    // Signed: with three or more queues the pairwise overlaps can add up to
    // more than the total, and the formula then goes negative.
    out->eff_s = ((double)total - (double)overlap) * 1e-9;
    out->elapsed_s = elapsed_s;
    if (elapsed_s > 0) {
        out->device_pct = 100.0 * out->eff_s / elapsed_s;
        out->host_pct = 100.0 - out->device_pct;
    }

    std::vector<uint32_t> present;
    for (uint32_t i = 0; i < nn; ++i)
        if (cnt[i])
            present.push_back(i);
    std::sort(present.begin(), present.end(), [&](uint32_t a, uint32_t b) {
        if (sum[a] != sum[b])
            return sum[a] > sum[b];
        return names[a] < names[b];
    });
    out->n_agg = (uint32_t)std::min<size_t>(present.size(), RNGX_PROF_MAX_AGG);
    for (uint32_t i = 0; i < out->n_agg; ++i) {
        rngx_prof_agg &g = out->agg[i];
        std::snprintf(g.name, sizeof g.name, "%s", names[present[i]].c_str());
        g.count = cnt[present[i]];
        g.abs_s = sum[present[i]] * 1e-9;
        g.rel_pct = total ? 100.0 * (double)sum[present[i]] / (double)total : 0.0;
    }

    struct Ov {
        uint32_t a, b;
        uint64_t ns;
    };
    std::vector<Ov> ovs;
    for (const auto &kv : pair_ns) {
        uint32_t a = kv.first.first, b = kv.first.second;
        // Name of smaller aggregate time first (ties: by name).
        if (sum[b] < sum[a] || (sum[b] == sum[a] && names[b] < names[a]))
            std::swap(a, b);
        ovs.push_back({a, b, kv.second});
    }
    std::sort(ovs.begin(), ovs.end(), [&](const Ov &p, const Ov &q) {
        if (p.ns != q.ns)
            return p.ns > q.ns;
        if (names[p.a] != names[q.a])
            return names[p.a] < names[q.a];
        return names[p.b] < names[q.b];
    });
    out->n_overlap = (uint32_t)std::min<size_t>(ovs.size(), RNGX_PROF_MAX_OVERLAP);
    for (uint32_t i = 0; i < out->n_overlap; ++i) {
        std::snprintf(out->overlap[i].name1, RNGX_PROF_NAME, "%s", names[ovs[i].a].c_str());
        std::snprintf(out->overlap[i].name2, RNGX_PROF_NAME, "%s", names[ovs[i].b].c_str());
        out->overlap[i].overlap_s = ovs[i].ns * 1e-9;
    }
    return RNGX_OK;
}

static void appendf(std::string &s, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    s += buf;
}

// Text summary with the table layout of Fig. 3.
static std::string format_summary(const rngx_prof_stats &st)
{
    const char *rule = "   ------------------------------------------------------------------\n";
    std::string s;
    s += " Aggregate times by event  :\n";
    s += rule;
    s += "   | Event name                     | Rel. time (%) | Abs. time (s) |\n";
    s += rule;
    for (uint32_t i = 0; i < st.n_agg; ++i)
        appendf(s, "   | %-30.30s | %13.4f | %13.4e |\n", st.agg[i].name, st.agg[i].rel_pct,
                st.agg[i].abs_s);
    s += rule;
    appendf(s, "                                    |         Total | %13.4e |\n", st.total_s);
    s += "                                    ---------------------------------\n";
    if (st.n_overlap) {
        s += " Event overlaps            :\n";
        s += rule;
        s += "   | Event 1                | Event 2                | Overlap (s)  |\n";
        s += rule;
        for (uint32_t i = 0; i < st.n_overlap; ++i)
            appendf(s, "   | %-22.22s | %-22.22s | %12.4e |\n", st.overlap[i].name1,
                    st.overlap[i].name2, st.overlap[i].overlap_s);
        s += rule;
        appendf(s, "                            |                  Total | %12.4e |\n",
                st.overlap_s);
        s += "                            -----------------------------------------\n";
    }
    appendf(s, " Tot. of all events (eff.) : %es\n", st.eff_s);
    appendf(s, " Total elapsed time        : %es\n", st.elapsed_s);
    appendf(s, " Time spent in device      : %.2f%%\n", st.device_pct);
    appendf(s, " Time spent in host        : %.2f%%\n", st.host_pct);
    if (st.n_dropped)
        appendf(s, " Events not logged (log full): %llu\n", (unsigned long long)st.n_dropped);
    return s;
}

namespace prof {
namespace {

// Tokens: window number << 16 | record index (the log holds at most 2^16).
constexpr size_t kMaxRecs = 1u << 16;

struct Rec {
    uint32_t name;
    hipStream_t stream;
    hipEvent_t ev0, ev1;
    bool ended; // end() recorded ev1 (an operation that failed to launch never ends)
};

struct State {
    std::mutex mu;
    bool enabled = true;
    bool open = false;
    std::vector<std::string> names;
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t ref = nullptr;
    std::chrono::steady_clock::time_point t0, t1;
    uint64_t dropped = 0;
    size_t cap = kMaxRecs;
    std::string summary;
    // Resolved rows of the last closed window.
    std::vector<EventRow> rows;
    bool resolved = false;
    // Window number (low 15 bits), carried in tokens so that an end() for a
    // record of an earlier window is ignored.
    uint32_t gen = 0;
};


State &S()
{
    static State *s = new State; // never destroyed: HIP may be gone at exit
    return *s;
}

uint32_t name_id(State &st, const char *name)
{
    for (uint32_t i = 0; i < st.names.size(); ++i)
        if (st.names[i] == name)
            return i;
    st.names.emplace_back(name);
    return (uint32_t)st.names.size() - 1;
}

hipError_t take_event(State &st, hipEvent_t *ev)
{
    if (!st.pool.empty()) {
        *ev = st.pool.back();
        st.pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(ev);
}

void recycle(State &st)
{
    for (Rec &r : st.recs) {
        st.pool.push_back(r.ev0);
        st.pool.push_back(r.ev1);
    }
    st.recs.clear();
    st.rows.clear();
    st.resolved = false;
    st.gen = (st.gen + 1) & 0x7fffu;
}

// Wait until every ended record's end event has completed.
int sync_ended(State &st)
{
    for (Rec &r : st.recs)
        if (r.ended)
            RNGX_HIP(hipEventSynchronize(r.ev1));
    return RNGX_OK;
}

// Wait for the logged work, stop the clock, resolve events to rows.
int close_locked(State &st)
{
    if (st.open) {
        int rc = sync_ended(st);
        if (rc)
            return rc;
        st.t1 = std::chrono::steady_clock::now();
        st.open = false;
    }
    if (!st.resolved) {
        // Records ended after the window closed are resolved too.
        int rc = sync_ended(st);
        if (rc)
            return rc;
        st.rows.clear();
        std::vector<int64_t> starts(st.recs.size());
        std::vector<uint64_t> durs(st.recs.size());
        int64_t lo = 0;
        for (size_t i = 0; i < st.recs.size(); ++i) {
            if (!st.recs[i].ended)
                continue;
            float ms0 = 0.f, msd = 0.f;
            RNGX_HIP(hipEventElapsedTime(&ms0, st.ref, st.recs[i].ev0));
            RNGX_HIP(hipEventElapsedTime(&msd, st.recs[i].ev0, st.recs[i].ev1));
            starts[i] = (int64_t)((double)ms0 * 1e6 + (ms0 >= 0 ? 0.5 : -0.5));
            durs[i] = msd > 0 ? (uint64_t)((double)msd * 1e6 + 0.5) : 0u;
            lo = std::min(lo, starts[i]);
        }
        for (size_t i = 0; i < st.recs.size(); ++i) {
            if (!st.recs[i].ended)
                continue;
            EventRow row;
            row.name = st.recs[i].name;
            row.queue = (uint64_t)(uintptr_t)st.recs[i].stream;
            row.start_ns = (uint64_t)(starts[i] - lo);
            row.end_ns = row.start_ns + durs[i];
            st.rows.push_back(row);
        }
        st.resolved = true;
    }
    return RNGX_OK;
}

} // namespace

int begin(const char *name, hipStream_t s)
{
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    if (!st.enabled || !st.open)
        return -1;
    if (st.recs.size() >= st.cap) {
        ++st.dropped;
        return -1;
    }
    Rec r;
    r.name = name_id(st, name);
    r.stream = s;
    r.ended = false;
    if (take_event(st, &r.ev0) != hipSuccess)
        return -1;
    if (take_event(st, &r.ev1) != hipSuccess) {
        st.pool.push_back(r.ev0);
        return -1;
    }
    if (hipEventRecord(r.ev0, s) != hipSuccess) {
        st.pool.push_back(r.ev0);
        st.pool.push_back(r.ev1);
        return -1;
    }
    st.recs.push_back(r);
    st.resolved = false;
    return (int)((st.gen << 16) | (uint32_t)(st.recs.size() - 1));
}

hipEvent_t end_event(int token, hipStream_t s)
{
    if (token < 0)
        return nullptr;
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    const uint32_t gen = (uint32_t)token >> 16, idx = (uint32_t)token & 0xffffu;
    if (gen != st.gen || idx >= st.recs.size() || st.recs[idx].ended)
        return nullptr; // a record of an earlier window
    if (hipEventRecord(st.recs[idx].ev1, s) != hipSuccess)
        return nullptr;
    st.recs[idx].ended = true;
    st.resolved = false;
    return st.recs[idx].ev1;
}

void end(int token, hipStream_t s) { (void)end_event(token, s); }

int start(hipStream_t ref_stream)
{
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    // Events of the previous window may still be pending; wait before reuse.
    (void)sync_ended(st);
    recycle(st);
    st.dropped = 0;
    if (!st.ref)
        RNGX_HIP(hipEventCreate(&st.ref));
    RNGX_HIP(hipEventRecord(st.ref, ref_stream));
    st.t0 = std::chrono::steady_clock::now();
    st.open = true;
    return RNGX_OK;
}

int stop()
{
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    if (!st.ref)
        return set_error(RNGX_E_NOINIT, "profiling window was never opened");
    return close_locked(st);
}

void release_all()
{
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    (void)sync_ended(st);
    recycle(st);
    for (hipEvent_t e : st.pool)
        RNGX_NOTE(hipEventDestroy(e));
    st.pool.clear();
    if (st.ref)
        RNGX_NOTE(hipEventDestroy(st.ref));
    st.ref = nullptr;
    st.open = false;
    st.names.clear();
    st.summary.clear();
}

int stats(rngx_prof_stats *out)
{
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    if (!st.ref)
        return set_error(RNGX_E_NOINIT, "profiling window was never opened");
    int rc = close_locked(st);
    if (rc)
        return rc;
    const double elapsed = std::chrono::duration<double>(st.t1 - st.t0).count();
    rc = analyze_rows(st.rows, st.names, elapsed, out);
    if (rc)
        return rc;
    out->n_dropped = st.dropped;
    return RNGX_OK;
}

const char *summary()
{
    rngx_prof_stats s;
    if (stats(&s) != RNGX_OK)
        return nullptr;
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    st.summary = format_summary(s);
    return st.summary.c_str();
}

int events(rngx_prof_event *out, uint32_t cap, uint32_t *n_out)
{
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    if (!st.ref)
        return set_error(RNGX_E_NOINIT, "profiling window was never opened");
    int rc = close_locked(st);
    if (rc)
        return rc;
    if (n_out)
        *n_out = (uint32_t)st.rows.size();
    if (cap && !out)
        return set_error(RNGX_E_INVAL, "events: NULL output with cap > 0");
    for (uint32_t i = 0; i < cap && i < st.rows.size(); ++i) {
        std::snprintf(out[i].name, RNGX_PROF_NAME, "%s", st.names[st.rows[i].name].c_str());
        out[i].queue = st.rows[i].queue;
        out[i].start_ns = st.rows[i].start_ns;
        out[i].end_ns = st.rows[i].end_ns;
    }
    return RNGX_OK;
}

int enable(int on)
{
    State &st = S();
    std::lock_guard<std::mutex> lk(st.mu);
    st.enabled = on != 0;
    return RNGX_OK;
}

} // namespace prof

int analyze_table(const rngx_prof_event *events, uint32_t n, double elapsed_s,
                  rngx_prof_stats *out)
{
    if (!out)
        return set_error(RNGX_E_INVAL, "analyze: NULL stats");
    if (n && !events)
        return set_error(RNGX_E_INVAL, "analyze: NULL events with n > 0");
    std::vector<std::string> names;
    std::vector<EventRow> rows(n);
    for (uint32_t i = 0; i < n; ++i) {
        char nm[RNGX_PROF_NAME + 1];
        std::memcpy(nm, events[i].name, RNGX_PROF_NAME);
        nm[RNGX_PROF_NAME] = 0;
        uint32_t id = 0;
        while (id < names.size() && names[id] != nm)
            ++id;
        if (id == names.size())
            names.emplace_back(nm);
        rows[i] = {id, events[i].queue, events[i].start_ns, events[i].end_ns};
    }
    return analyze_rows(rows, names, elapsed_s, out);
}

std::string summary_of(const rngx_prof_stats &st) { return format_summary(st); }

namespace {

// The event name with a terminating NUL; control characters become '_' so
// a name can never break a line of the table.
std::string clean_name(const char *raw)
{
    std::string s(raw, strnlen(raw, RNGX_PROF_NAME));
    for (char &ch : s)
        if ((unsigned char)ch < 0x20 || ch == 0x7f)
            ch = '_';
    return s;
}

void json_string(FILE *f, const std::string &s)
{
    std::fputc('"', f);
    for (char ch : s) {
        if (ch == '"' || ch == '\\')
            std::fputc('\\', f);
        std::fputc(ch, f);
    }
    std::fputc('"', f);
}

} // namespace

int write_table(const rngx_prof_event *events, uint32_t n, const char *path, int format)
{
    if (!path)
        return set_error(RNGX_E_INVAL, "profile export: NULL path");
    if (n && !events)
        return set_error(RNGX_E_INVAL, "profile export: NULL events with n > 0");
    if (format != RNGX_EXPORT_TABLE && format != RNGX_EXPORT_TRACE)
        return set_error(RNGX_E_INVAL, "profile export: unknown format %d", format);
    for (uint32_t i = 0; i < n; ++i)
        if (events[i].end_ns < events[i].start_ns)
            return set_error(RNGX_E_INVAL, "profile export: event %u ends before it starts", i);
    // Events by start time; queues numbered in order of their first event.
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return events[a].start_ns < events[b].start_ns;
    });
    std::vector<uint64_t> queues;
    std::vector<uint32_t> qidx(n);
    for (uint32_t i : order) {
        uint32_t q = 0;
        while (q < queues.size() && queues[q] != events[i].queue)
            ++q;
        if (q == queues.size())
            queues.push_back(events[i].queue);
        qidx[i] = q;
    }
    FILE *f = std::fopen(path, "w");
    if (!f)
        return set_error(RNGX_E_INVAL, "profile export: cannot open %s: %s", path,
                         std::strerror(errno));
    if (format == RNGX_EXPORT_TABLE) {
        std::fprintf(f, "queue\tt_start\tt_end\tevent\n");
        for (uint32_t i : order)
            std::fprintf(f, "q%u\t%llu\t%llu\t%s\n", qidx[i],
                         (unsigned long long)events[i].start_ns,
                         (unsigned long long)events[i].end_ns,
                         clean_name(events[i].name).c_str());
    } else {
        std::fprintf(f, "{\"displayTimeUnit\": \"ns\", \"traceEvents\": [");
        bool first = true;
        for (uint32_t q = 0; q < queues.size(); ++q) {
            std::fprintf(f, "%s\n{\"name\": \"thread_name\", \"ph\": \"M\", \"pid\": 1, "
                            "\"tid\": %u, \"args\": {\"name\": \"q%u\"}}",
                         first ? "" : ",", q, q);
            first = false;
        }
        for (uint32_t i : order) {
            std::fprintf(f, "%s\n{\"name\": ", first ? "" : ",");
            json_string(f, clean_name(events[i].name));
            std::fprintf(f, ", \"cat\": \"rngx\", \"ph\": \"X\", \"pid\": 1, \"tid\": %u, "
                            "\"ts\": %.3f, \"dur\": %.3f}",
                         qidx[i], events[i].start_ns / 1e3,
                         (events[i].end_ns - events[i].start_ns) / 1e3);
            first = false;
        }
        std::fprintf(f, "\n]}\n");
    }
    const bool ok = !std::ferror(f);
    if (std::fclose(f) != 0 || !ok)
        return set_error(RNGX_E_INVAL, "profile export: cannot write %s", path);
    return RNGX_OK;
}

} // namespace rngx
