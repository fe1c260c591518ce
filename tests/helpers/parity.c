/*
 * parity.c -- multi-threaded element-wise comparison of device outputs (after
 * their copy to host memory) with the CPU oracle. Test infrastructure: it
 * calls only the oracle's entry points (oracle/oracle.c) and compares bytes;
 * it computes nothing of the generator itself.
 *
 * The outputs checked here are gigabytes long, so the oracle's values are
 * produced a tile at a time into a small per-thread buffer (a few hundred
 * KiB, cache-resident) with oracle_emit_rows, which continues the plain loop
 * from a caller-held state array, and each tile is compared with memcmp.
 * Host threads split the work by work-item (plain output: each thread owns
 * a contiguous slice of columns and its slice of the state array) or by
 * request (batched and served output).
 *
 * Every function returns the number of mismatching values and the first
 * mismatch (lowest row, then lowest column; or lowest request, then lowest
 * value index), plus the number of zero states the oracle met (the
 * never-zero invariant says 0).
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The oracle (liboracle.so). */
uint64_t oracle_value(uint64_t seed, uint32_t gid, uint64_t k);
void oracle_seed_range(uint64_t seed, uint32_t g0, uint64_t count, uint64_t cursor,
                       uint64_t *st);
uint64_t oracle_emit_rows(uint64_t *st, uint64_t count, uint32_t n_rows, int word, void *out,
                          uint64_t ld);

typedef struct {
    uint64_t mismatches;
    uint64_t first_a; /* row, or request */
    uint64_t first_b; /* column, or value index within the request */
    uint64_t zeros;
    int32_t failed;   /* a thread could not allocate its buffer */
    int32_t reserved;
} pc_result;

/* Same layout as the oracle's request record. */
typedef struct {
    uint64_t seed;
    uint64_t offset;
    uint64_t length;
    uint32_t gid;
    uint32_t reserved;
} pc_req;

static size_t word_size(int word) { return (word == 1 || word == 3) ? 4u : 8u; }

static void note(pc_result *r, uint64_t a, uint64_t b)
{
    if (r->mismatches == 0 || a < r->first_a || (a == r->first_a && b < r->first_b)) {
        r->first_a = a;
        r->first_b = b;
    }
    r->mismatches++;
}

static void merge(pc_result *into, const pc_result *r)
{
    if (r->mismatches) {
        if (!into->mismatches || r->first_a < into->first_a ||
            (r->first_a == into->first_a && r->first_b < into->first_b)) {
            into->first_a = r->first_a;
            into->first_b = r->first_b;
        }
        into->mismatches += r->mismatches;
    }
    into->zeros += r->zeros;
    into->failed |= r->failed;
}

/* Count the differing values of two equally long runs of words. */
static void diff_words(const char *exp, const char *got, uint64_t count, size_t es,
                       pc_result *r, uint64_t a, uint64_t b0)
{
    if (memcmp(exp, got, count * es) == 0)
        return;
    for (uint64_t t = 0; t < count; ++t)
        if (memcmp(exp + t * es, got + t * es, es) != 0)
            note(r, a, b0 + t);
}

/* ---- plain output ------------------------------------------------------- */

typedef struct {
    const char *got;   /* row 0, column 0 */
    uint64_t ld;       /* row stride in words */
    uint64_t c0, c1;   /* this thread's columns */
    uint32_t n_rows;
    int word;
    uint64_t *st;      /* the whole state array (indexed by column) */
    pc_result res;
} plain_job;

static void *plain_worker(void *arg)
{
    plain_job *j = (plain_job *)arg;
    const size_t es = word_size(j->word);
    uint64_t tile = (256u * 1024u) / ((uint64_t)j->n_rows * es);
    if (tile < 64)
        tile = 64;
    char *buf = (char *)malloc((size_t)tile * j->n_rows * es);
    if (!buf) {
        j->res.failed = 1;
        return NULL;
    }
    for (uint64_t c = j->c0; c < j->c1; c += tile) {
        const uint64_t cnt = (j->c1 - c) < tile ? (j->c1 - c) : tile;
        j->res.zeros += oracle_emit_rows(j->st + c, cnt, j->n_rows, j->word, buf, cnt);
        for (uint32_t k = 0; k < j->n_rows; ++k)
            diff_words(buf + (size_t)k * cnt * es, j->got + ((size_t)k * j->ld + c) * es, cnt,
                       es, &j->res, k, c);
    }
    free(buf);
    return NULL;
}

/* Compare n_rows rows of n words (row stride ld words) with the oracle
 * continuing from st[0..n) (advanced by n_rows steps on return). */
void pc_check_plain_rows(const void *got, uint64_t ld, uint64_t n, uint32_t n_rows, uint64_t *st,
                         int word, int threads, pc_result *out)
{
    memset(out, 0, sizeof *out);
    if (threads < 1)
        threads = 1;
    if ((uint64_t)threads > n)
        threads = n ? (int)n : 1;
    plain_job *jobs = (plain_job *)calloc((size_t)threads, sizeof *jobs);
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof *tid);
    int *ok = (int *)calloc((size_t)threads, sizeof *ok);
    if (!jobs || !tid || !ok) {
        out->failed = 1;
        free(jobs);
        free(tid);
        free(ok);
        return;
    }
    for (int t = 0; t < threads; ++t) {
        plain_job *j = &jobs[t];
        j->got = (const char *)got;
        j->ld = ld;
        j->c0 = n * (uint64_t)t / (uint64_t)threads;
        j->c1 = n * (uint64_t)(t + 1) / (uint64_t)threads;
        j->n_rows = n_rows;
        j->word = word;
        j->st = st;
    }
    for (int t = 1; t < threads; ++t)
        ok[t] = pthread_create(&tid[t], NULL, plain_worker, &jobs[t]) == 0;
    plain_worker(&jobs[0]);
    for (int t = 1; t < threads; ++t) {
        if (ok[t])
            pthread_join(tid[t], NULL);
        else
            plain_worker(&jobs[t]);
    }
    for (int t = 0; t < threads; ++t)
        merge(out, &jobs[t].res);
    free(jobs);
    free(tid);
    free(ok);
}

/* ---- seeding ------------------------------------------------------------ */

typedef struct {
    uint64_t seed, g0, count, cursor;
    uint64_t *st;
} seed_job;

static void *seed_worker(void *arg)
{
    seed_job *j = (seed_job *)arg;
    oracle_seed_range(j->seed, (uint32_t)j->g0, j->count, j->cursor, j->st);
    return NULL;
}

/* st[t] = value(seed, g0 + t, cursor) for t < count, over `threads` threads. */
void pc_seed_states(uint64_t seed, uint64_t g0, uint64_t count, uint64_t cursor, uint64_t *st,
                    int threads)
{
    if (threads < 1)
        threads = 1;
    seed_job *jobs = (seed_job *)calloc((size_t)threads, sizeof *jobs);
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof *tid);
    int *ok = (int *)calloc((size_t)threads, sizeof *ok);
    if (!jobs || !tid || !ok) {
        oracle_seed_range(seed, (uint32_t)g0, count, cursor, st);
        free(jobs);
        free(tid);
        free(ok);
        return;
    }
    for (int t = 0; t < threads; ++t) {
        const uint64_t a = count * (uint64_t)t / (uint64_t)threads;
        const uint64_t b = count * (uint64_t)(t + 1) / (uint64_t)threads;
        jobs[t] = (seed_job){seed, g0 + a, b - a, cursor, st + a};
    }
    for (int t = 1; t < threads; ++t)
        ok[t] = pthread_create(&tid[t], NULL, seed_worker, &jobs[t]) == 0;
    seed_worker(&jobs[0]);
    for (int t = 1; t < threads; ++t) {
        if (ok[t])
            pthread_join(tid[t], NULL);
        else
            seed_worker(&jobs[t]);
    }
    free(jobs);
    free(tid);
    free(ok);
}

/* ---- batched and served output ------------------------------------------ */

typedef struct {
    const pc_req *reqs;
    uint32_t m;
    const char *got;
    const uint64_t *bases;  /* got index of each request's first value */
    const uint64_t *starts; /* optional: state at each request's offset */
    int word;
    uint32_t *next;         /* shared request counter */
    pc_result res;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *j = (batch_job *)arg;
    const size_t es = word_size(j->word);
    const uint64_t tile = 32768;
    char *buf = (char *)malloc((size_t)tile * es);
    if (!buf) {
        j->res.failed = 1;
        return NULL;
    }
    for (;;) {
        const uint32_t r = __atomic_fetch_add(j->next, 1u, __ATOMIC_RELAXED);
        if (r >= j->m)
            break;
        const pc_req *q = &j->reqs[r];
        uint64_t x = j->starts ? j->starts[r] : oracle_value(q->seed, q->gid, q->offset);
        const char *g = j->got + (size_t)j->bases[r] * es;
        for (uint64_t t = 0; t < q->length; t += tile) {
            const uint64_t cnt = (q->length - t) < tile ? (q->length - t) : tile;
            /* One stream, continued: a single state emitted cnt times. */
            j->res.zeros += oracle_emit_rows(&x, 1, (uint32_t)cnt, j->word, buf, 1);
            diff_words(buf, g + (size_t)t * es, cnt, es, &j->res, r, t);
        }
    }
    free(buf);
    return NULL;
}

/* Compare m requests with the oracle: request r's values are
 * value(seed_r, gid_r, offset_r + t), t < length_r, found at got[bases[r] + t].
 * With `starts`, starts[r] is taken as the state at offset_r (the caller
 * derives it); otherwise the oracle steps there from the initial state. */
void pc_check_requests(const pc_req *reqs, uint32_t m, const void *got, const uint64_t *bases,
                       const uint64_t *starts, int word, int threads, pc_result *out)
{
    memset(out, 0, sizeof *out);
    if (threads < 1)
        threads = 1;
    if ((uint32_t)threads > m)
        threads = m ? (int)m : 1;
    uint32_t next = 0;
    batch_job *jobs = (batch_job *)calloc((size_t)threads, sizeof *jobs);
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof *tid);
    int *ok = (int *)calloc((size_t)threads, sizeof *ok);
    if (!jobs || !tid || !ok) {
        out->failed = 1;
        free(jobs);
        free(tid);
        free(ok);
        return;
    }
    for (int t = 0; t < threads; ++t)
        jobs[t] = (batch_job){reqs, m, (const char *)got, bases, starts, word, &next, {0}};
    for (int t = 1; t < threads; ++t)
        ok[t] = pthread_create(&tid[t], NULL, batch_worker, &jobs[t]) == 0;
    batch_worker(&jobs[0]);
    for (int t = 1; t < threads; ++t)
        if (ok[t])
            pthread_join(tid[t], NULL);
    for (int t = 0; t < threads; ++t)
        merge(out, &jobs[t].res);
    free(jobs);
    free(tid);
    free(ok);
}
