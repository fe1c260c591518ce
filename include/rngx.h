/*
 * rngx.h -- C ABI of an MI355X (gfx950) implementation of the massive
 * pseudo-random number generator in the example application of "cf4ocl: a C
 * framework for OpenCL" (Section 5, "Example: massive pseudo-random number
 * generator"; supplementary Listings S4 and S5).
 *
 * What is computed (all arithmetic exact, unsigned, wrapping):
 *   J(a)  the six-round 32-bit integer hash of Listing S4 ("low bits"),
 *   W(a)  the five-round shift-multiply hash of Listing S4 ("high bits"),
 *   H(s, g) = (W(low ^ h) << 32) | low,  low = J(g ^ l),
 *            l = J(lo32 s) ^ J(0),  h = W(hi32 s) ^ W(0)
 *         the initial state of work-item g under a 64-bit seed s; s = 0 gives
 *         exactly the paper's init kernel (low = J(g), high = W(low)); the
 *         all-zero state, reachable for one (s, g) pair when s != 0, is
 *         replaced by W(0) << 32,
 *   XS(x) one step of the 64-bit xorshift of Listing S5: x ^= x << 21;
 *         x ^= x >> 35; x ^= x << 4,
 *   V(s, g, k) = XS^k(H(s, g)), value number k of work-item g's stream.
 * The values written by the init kernel are the first batch of output
 * (Section 5), so value number 0 of every stream is its initial state.
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status (RNGX_OK or a negative RNGX_E_*
 *    code) unless stated otherwise. On failure, rngx_last_error() returns a
 *    message for the calling thread (the paper's error-object convention,
 *    Section 4.1). The library never exits the process.
 *  - One process-wide generator context, guarded by a mutex; calls from
 *    several host threads are serialised.
 *  - Device pointers are plain HIP device addresses on the current device.
 *    `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *    Work is enqueued asynchronously on `stream`; the library orders its own
 *    use of the generator state across streams with HIP events.
 *  - The caller owns every buffer it passes and must keep it alive until the
 *    enqueued work has completed. The library owns its state buffer, events
 *    and the text it returns.
 */
#ifndef RNGX_H
#define RNGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define RNGX_OK 0
#define RNGX_E_INVAL (-1)  /* invalid argument (NULL, misaligned, 0 states, overflow) */
#define RNGX_E_NOINIT (-2) /* generator used before rngx_init */
#define RNGX_E_HIP (-3)    /* HIP runtime error; rngx_last_error() holds its text */
#define RNGX_E_NOMEM (-4)  /* device allocation failed */
#define RNGX_E_BUSY (-5)   /* resource temporarily full; retry later */
#define RNGX_E_ABORTED (-6) /* a caller-supplied consumer asked to stop */

/* ------------------------------------------------------------------------ */
/* Generator lifecycle                                                       */
/* ------------------------------------------------------------------------ */

/* Seed n_states streams: state[g] = H(seed, g) for g < n_states (Listing S4;
 * Section 5, the init kernel). Allocates the library-owned state buffer
 * (8 * n_states bytes of device memory) on the current device, launches the
 * init kernel on the library's own stream, resets the cursor to 0 and
 * restarts the profiler (as the paper starts profiling just before init).
 * Calling it again releases the previous state first.
 * Errors: RNGX_E_INVAL if n_states == 0 (n_states is a 32-bit count, as the
 * paper's nseeds is a cl_uint); RNGX_E_NOMEM; RNGX_E_HIP. */
int rngx_init(uint64_t seed, uint32_t n_states);

/* Produce the next n_iters iterations of every stream (Section 5: each rng
 * kernel invocation advances every state once; Eq. 1: 8 * n * i bytes):
 *     out[k * n_states + g] = V(seed, g, cursor + k),  k < n_iters,
 * iteration-major, i.e. the byte order the paper's program writes to its
 * standard output; then cursor += n_iters.
 * out: device memory of at least 8 * n_states * n_iters bytes, 8-byte
 *      aligned (16-byte alignment and an even n_states give the fastest
 *      stores). n_iters == 0 is a successful no-op.
 * Errors: RNGX_E_NOINIT; RNGX_E_INVAL (out NULL or misaligned, the byte
 * count overflows size_t, or the cursor would pass value number 2^64 - 1);
 * RNGX_E_HIP. */
int rngx_generate(uint32_t n_iters, uint64_t *out, void *stream);

/* As rngx_generate, writing the low 32 bits of each value:
 *     out[k * n_states + g] = (uint32_t)V(seed, g, cursor + k).
 * It advances the same cursor. out must be 4-byte aligned. */
int rngx_generate_u32(uint32_t n_iters, uint32_t *out, void *stream);

/* Current generator parameters (any pointer may be NULL).
 * Errors: RNGX_E_NOINIT. */
int rngx_info(uint64_t *seed, uint32_t *n_states, uint64_t *cursor);

/* Checkpoint of the plain generator. Between generate calls the whole
 * generator is its n_states 64-bit states plus the seed and the cursor: the
 * state of work-item g is V(seed, g, cursor), the next value it emits (the
 * rng kernel of Section 5 likewise keeps it in a buffer between launches).
 * rngx_get_state waits for all queued work that uses the state, then copies
 * the states into `states` (host memory, n entries, caller-owned) and
 * returns seed and cursor (either pointer may be NULL).
 * Errors: RNGX_E_NOINIT; RNGX_E_INVAL (states NULL, or n != n_states);
 * RNGX_E_HIP. */
int rngx_get_state(uint64_t *states, uint32_t n, uint64_t *seed, uint64_t *cursor);

/* Resume from a checkpoint: replaces the generator (as rngx_init does, on
 * the current device) by the n states read from `states` (host memory,
 * copied before the call returns), labelled with `seed` and `cursor`.
 * Generation then continues exactly where the checkpointed generator
 * stopped. Starts a new profiling window, like rngx_init.
 * Errors: RNGX_E_INVAL (states NULL, n == 0, or a state equal to 0, which
 * xorshift maps to itself and no seeding produces); RNGX_E_NOMEM;
 * RNGX_E_HIP. */
int rngx_set_state(uint64_t seed, const uint64_t *states, uint32_t n, uint64_t cursor);

/* Release the state buffer, events, streams and every other resource the
 * library holds (the constructor/destructor discipline of Section 4.1).
 * Safe to call when nothing is initialised. */
int rngx_shutdown(void);

/* Message describing the calling thread's last failure ("" if none). */
const char *rngx_last_error(void);

/* Static name of a status code (the paper's errors module, Section 4.4). */
const char *rngx_strerror(int code);

/* HIP errors that no call could return (the paper reports every error to
 * the caller, Section 4.1; these are the ones with no caller left to
 * receive them). Two kinds are recorded, each with the place it was met,
 * the HIP error name and the host thread:
 *  - "released": a HIP call of the library's own release paths failed
 *    (freeing buffers, destroying streams, events and graphs, the waits
 *    before them) inside a call that still succeeded or was already
 *    failing for another reason;
 *  - "stray": an error was pending in the calling thread when the library
 *    was about to launch a kernel, left by an earlier HIP call that is not
 *    the library's (every library call consumes the status of its own HIP
 *    calls); it is recorded and cleared, so that the launch reports only
 *    its own status.
 * *released and *stray (either may be NULL) receive the counts since the
 * last clear; text (may be NULL) receives up to cap - 1 bytes of the most
 * recent notes (at most 32, one per line, oldest first), NUL-terminated.
 * clear != 0 resets counts and notes after reading them.
 * Errors: RNGX_E_INVAL if text is non-NULL and cap == 0. */
int rngx_hip_notes(uint64_t *released, uint64_t *stray, char *text, size_t cap, int clear);

/* ------------------------------------------------------------------------ */
/* Launch configuration of the plain generator                               */
/* ------------------------------------------------------------------------ */

/* block: threads per block (64..1024, a multiple of 64), or 0 for the
 *        library's choice at each call (the other fields are then
 *        ignored).
 * chunks: 16-byte stores per lane per iteration (1, 2 or 4); a lane then
 *         owns 2*chunks (u64) or 4*chunks (u32) work-items, and every store
 *         instruction of a wavefront covers 1 KiB of contiguous output.
 * nontemporal: 1 to use non-temporal (streaming) stores.
 * pace_gbs: 0, or a row schedule for the launch, 1000..20000 (GB/s). With a
 *         schedule the kernel runs on a persistent grid of every block that
 *         fits on the device at once, the blocks walking strips of columns
 *         in turn, and every wavefront writes its iteration k of strip s
 *         no earlier than its own start time + (s * n_iters + k) times the
 *         time the resident wavefronts' share of a row takes at pace_gbs,
 *         read from the device's constant-rate clock. Wavefronts ahead of
 *         the schedule wait; those behind run freely, so the grid moves
 *         down the rows together instead of drifting apart (each wait is
 *         bounded; the schedule never changes a value). Used for calls of
 *         at least 2 iterations on 16-byte aligned rows; other calls run
 *         the unscheduled kernel.
 * Defaults: u64 block 512, 2 chunks, non-temporal stores, schedule 7000
 * GB/s; u32 block 0, the library's choice, which is the same launch
 * (measured on MI355X: 6.8-7.1 TB/s at every size from 2^20 to 2^26 states
 * x 256 iterations, u64 and u32, against 5.4-6.5 for the fastest
 * unscheduled launch, block 512 with 4 chunks; 7000 leaves a margin below
 * the rates where a schedule falls behind the device and loses its effect).
 * The autotuner (rngx_autotune_plain) picks among 88 configurations.
 * The output never depends on the configuration. */
typedef struct rngx_launch {
    uint32_t block;
    uint32_t chunks;
    uint32_t nontemporal;
    uint32_t pace_gbs;
} rngx_launch;

/* Set the configuration used by rngx_generate (u32 != 0: rngx_generate_u32).
 * Errors: RNGX_E_INVAL for values outside the ranges above. */
int rngx_set_launch(int u32, const rngx_launch *cfg);
int rngx_get_launch(int u32, rngx_launch *cfg);

/* Output scrambler (process-wide, kept across rngx_init): it applies to
 * rngx_generate, rngx_generate_u32, rngx_stream_to_host,
 * rngx_generate_batch and rngx_autotune_batch at each call, and to a
 * request server as set when rngx_serve_start ran. The paper
 * notes, discussing Fig. 5, that its generator kernels are much shorter
 * than the transfers, so a more complex generator would cost nothing.
 * RNGX_SCRAMBLE_NONE (default): the paper's generator, the state is the
 *   output (its low half for 32-bit output).
 * RNGX_SCRAMBLE_STAR: the xorshift* construction (Vigna, 2016) on the same
 *   states: each output is the state times 2685821657736338717 modulo 2^64
 *   (its high half for 32-bit output). The states, the cursor, seeding,
 *   checkpoints, jump-ahead and the served cursors are unchanged.
 * Errors: RNGX_E_INVAL for an unknown scrambler or a NULL pointer. */
#define RNGX_SCRAMBLE_NONE 0
#define RNGX_SCRAMBLE_STAR 1
int rngx_set_scrambler(int scrambler);
int rngx_get_scrambler(int *scrambler);

/* ------------------------------------------------------------------------ */
/* Streaming to host memory (Section 5, Fig. 2)                              */
/* ------------------------------------------------------------------------ */

/* Host-side consumer of one streamed step: `values` points at the step's
 * host slot (bytes = iters_per_step * n_states * element size), `step` is
 * its index from 0. It runs on the thread that called rngx_stream_to_host,
 * in step order. Return 0 to continue, non-zero to stop the stream. It may
 * call rngx functions; generate calls made from it advance the same cursor. */
typedef int (*rngx_consume_fn)(void *user, uint64_t step, const void *values, size_t bytes);

/* Stream n_steps * iters_per_step iterations to host memory with generation
 * and device-to-host copies overlapped on two streams (Section 5: the init
 * and rng kernels run on one command queue, the reads on a second one, with
 * device-side double buffering).
 * Step k generates iters_per_step iterations (exactly as rngx_generate /
 * rngx_generate_u32 would, continuing the cursor) into device buffer k % 2
 * (dev0 or dev1, each of dev_bytes bytes) on gen_stream, then copies them to
 * host slot k % host_slots of `host` on copy_stream. Step k's generation
 * waits only for the copy of step k - 2; step k's copy waits for its
 * generation. Kernels are profiled as RNG_KERNEL and copies as READ_BUFFER.
 * host: host_slots consecutive slots of one step each; page-locked memory
 *       (hipHostMalloc, or torch pin_memory) makes the copies asynchronous
 *       and lets the copy kernel write it directly (see rngx_set_copy_mode).
 * consume: optional (NULL = no host consumer, as when the paper's output is
 *       sent to the null device); with it, a slot is refilled only after the
 *       consumer returned for the step it held.
 * gen_stream, copy_stream: distinct streams, or NULL for the library's own
 *       pair. The call returns when every copy has completed (and every
 *       step has been consumed); on an error or a stop it first waits for
 *       all the work it enqueued on both streams, so no kernel or copy
 *       still uses the buffers when it returns.
 * Errors: RNGX_E_NOINIT; RNGX_E_INVAL (NULL/equal/misaligned buffers, a
 * step larger than dev_bytes, host_slots == 0, equal streams);
 * RNGX_E_ABORTED when the consumer stops the stream (steps generated so far
 * have advanced the cursor); RNGX_E_HIP. */
int rngx_stream_to_host(uint32_t n_steps, uint32_t iters_per_step, int u32, void *dev0,
                        void *dev1, size_t dev_bytes, void *host, uint32_t host_slots,
                        rngx_consume_fn consume, void *user, void *gen_stream,
                        void *copy_stream);

/* Test hook for the pipeline's error path. In the paper's example a failed
 * read ends the communications thread, which first wakes the main thread;
 * the main thread then sees the error and stops (Section 5; supplementary
 * Listings S1 and S2). Here, in the next rngx_stream_to_host call, the copy
 * of step `step` fails before it is enqueued: the call waits for everything
 * it already enqueued on both streams, calls the consumer for no further
 * step, and returns RNGX_E_HIP with a message naming the step. Steps up to
 * and including `step` have been generated (the cursor has advanced past
 * them); the consumer has received the steps whose slots were already
 * recycled. The hook fires once; UINT64_MAX disarms it. Nothing fails on the
 * device: no kernel is launched for the failing copy.
 * Errors: none. */
int rngx_inject_copy_failure(uint64_t step);

/* How rngx_stream_to_host moves each step to the host:
 * RNGX_COPY_KERNEL (default): the library's copy kernel stores straight into
 *   the page-locked host buffer through its device-mapped address (falls
 *   back to RNGX_COPY_RUNTIME if `host` is not page-locked memory);
 * RNGX_COPY_RUNTIME: hipMemcpyAsync on the copy stream.
 * blocks: workgroups of 256 lanes for the copy kernel (1..65536, default 16).
 * Errors: RNGX_E_INVAL for an unknown mode or blocks out of range. */
#define RNGX_COPY_KERNEL 0
#define RNGX_COPY_RUNTIME 1
int rngx_set_copy_mode(int mode, uint32_t blocks);
int rngx_get_copy_mode(int *mode, uint32_t *blocks);

/* ------------------------------------------------------------------------ */
/* Batched ragged streams                                                    */
/* ------------------------------------------------------------------------ */

/* One request: `length` consecutive values of the stream of work-item `gid`
 * under `seed`, starting at value number `offset`, i.e.
 * V(seed, gid, offset + t) for t < length. 32 bytes, host memory. */
typedef struct rngx_req {
    uint64_t seed;
    uint64_t offset;
    uint64_t length;
    uint32_t gid;
    uint32_t reserved; /* must be 0 */
} rngx_req;

/* Generate m independent streams of uneven lengths in one launch:
 *     out[base_j + t] = V(seed_j, gid_j, offset_j + t),  t < length_j,
 *     base_j = length_0 + ... + length_{j-1}  (packed in request order).
 * The paper's init and rng kernels give one uniform grid of streams; here
 * every request is its own seeded stream, started at any value number by
 * GF(2) jump-ahead (so long streams split across many wavefronts), all in
 * one persistent kernel launch, replayed from a captured HIP graph when the
 * graph mode of the batch configuration is on. Independent of rngx_init:
 * the plain generator's state and cursor are untouched.
 * reqs: m requests in host memory (zero-length requests produce nothing).
 * out:  device memory of out_cap uint64 values, 16-byte aligned.
 * Errors: RNGX_E_INVAL (NULL reqs with m > 0, NULL or misaligned out, a
 * nonzero reserved field, a request running past value number 2^64 - 1
 * (offset + length > 2^64), total length above out_cap or overflowing);
 * RNGX_E_NOMEM; RNGX_E_HIP. */
int rngx_generate_batch(const rngx_req *reqs, uint32_t m, uint64_t *out, uint64_t out_cap,
                        void *stream);

/* For callers that cannot allocate (code that must not call hipMalloc:
 * under HIP graph capture, tight serving loops, harnesses that forbid it):
 * the same output as rngx_generate_batch, from a call that allocates
 * nothing. The request table goes to a static device array of the library
 * (262,272 bytes, one per device, held until the process ends) instead of
 * a buffer allocated for the batch; the jump tables are static device arrays
 * too. The launch is direct (never a captured graph) in the batch
 * configuration's launch shape; no profiler events are recorded.
 * reqs, m, out, out_cap, stream: as rngx_generate_batch; at most
 * RNGX_NOALLOC_MAX_REQS requests. The table is copied from pageable host
 * memory, which HIP does synchronously, so the call may block until the
 * work already queued on `stream` has run; the kernel itself runs
 * asynchronously.
 * Every call on a device shares that device's table: calls that overlap on
 * one device (other threads, or other streams whose kernels are still
 * running) race. The first call on a device (or any earlier batched call
 * there) fills its jump tables and takes the table's device address:
 * set-up, once per device.
 * Errors: as rngx_generate_batch; RNGX_E_INVAL for m above
 * RNGX_NOALLOC_MAX_REQS, checked before any device work. */
#define RNGX_NOALLOC_MAX_REQS 4096u
int rngx_generate_batch_noalloc(const rngx_req *reqs, uint32_t m, uint64_t *out, uint64_t out_cap,
                                void *stream);

/* Launch configuration of the batched kernel.
 * values_per_lane: S, values each lane produces per work item (8, 16, 32,
 *   64, 128, 256, 512 or 1024); a work item is a tile of 64 * S output values.
 * waves_per_block: 1..4; blocks: 1..65536 (the persistent grid; 0 means 8
 *   waves per compute unit);
 * use_graph: 1 to capture the table upload and the launch in a HIP graph
 *   once and replay it, 0 to launch directly;
 * row_values: values each lane stages in LDS per round before the wave
 *   writes them out (8: 64-byte rows, 5 KiB of LDS per wave; 16: 128-byte
 *   rows, 9 KiB per wave; at most values_per_lane);
 * run_items: 0..64, most work items a wave takes at once (0 means 1;
 *   fewer near the end of the batch, down to 1); within a run, a wave
 *   moving to the next tile of the same request carries each lane's state
 *   forward instead of jumping from the stream's start;
 * per_item: 1 to launch one wave per work item instead (the grid is sized
 *   to the items, there is no work counter, blocks and run_items are
 *   ignored), 0 for the persistent grid.
 * group: 0, or the grouped scheduled order with groups of 16, 32, 64 or 128
 *   wavefronts (per_item must be 0; blocks and run_items are ignored). The
 *   grid is every block that fits on the device at once, rounded down to
 *   whole groups; the work items are cut into regions of group *
 *   group_steps consecutive items, group q takes regions q, q + Q, ... (Q
 *   groups), and at step s of a region its wavefront j takes item
 *   s * group + j, so a group's wavefronts write side by side and move
 *   through the region together; between steps of one request each lane
 *   carries its state group * 64 * S - S values on with one nibble-table
 *   product instead of a jump from the stream's start. Stores are
 *   non-temporal.
 * group_steps: 1..256 with a group (0 without).
 * pace_gbs: with a group, 0 or a row schedule of 1000..20000 GB/s: every
 *   wavefront takes its step k no earlier than its start time + k times the
 *   time the grid's items of one step take at pace_gbs, on the device's
 *   constant-rate clock (bounded waits, as for rngx_launch.pace_gbs). 0
 *   without a group.
 * Default: the grouped order with values_per_lane 16, 4 waves per block,
 * a graph, 16-value rows, groups of 32, 8 steps and 6250 GB/s (the
 * autotuner's pick on a 4,096-stream table on MI355X, 6.2 TB/s there
 * against 5.9 for the persistent grid with S = 256).
 * The output never depends on the configuration. */
typedef struct rngx_batch_cfg {
    uint32_t values_per_lane;
    uint32_t waves_per_block;
    uint32_t blocks;
    uint32_t use_graph;
    uint32_t row_values;
    uint32_t run_items;
    uint32_t per_item;
    uint32_t group;
    uint32_t group_steps;
    uint32_t pace_gbs;
} rngx_batch_cfg;

int rngx_set_batch_cfg(const rngx_batch_cfg *cfg);
int rngx_get_batch_cfg(rngx_batch_cfg *cfg);

#define RNGX_TUNE_MAX 128
typedef struct rngx_tune_entry {
    rngx_batch_cfg cfg;
    double ms; /* mean kernel time over the timed repetitions */
} rngx_tune_entry;
#define RNGX_TUNE_CONFIRM 4
typedef struct rngx_tune_result {
    rngx_batch_cfg best;
    double best_ms;  /* the best confirmation timing */
    double best_gbs; /* output bytes / best_ms */
    uint32_t n_tried;
    uint32_t reserved;
    rngx_tune_entry tried[RNGX_TUNE_MAX];
    /* The RNGX_TUNE_CONFIRM fastest candidates timed again with 3 * reps
     * launches each; best is the fastest of these. */
    rngx_tune_entry confirm[RNGX_TUNE_CONFIRM];
} rngx_tune_result;

/* Autotuner (the paper's work-size suggestion, Section 6.1, made empirical):
 * time every candidate configuration of the persistent launch
 * (values_per_lane 64..512 x waves_per_block 2 or 4 x run_items 1 or 8 x
 * 8, 16 or 32 waves per compute unit, those whose LDS fits; 16-value rows)
 * and of the grouped order (values_per_lane 16, 16-value rows, 4
 * wavefronts per block x groups of 16 or 32 wavefronts x 8 or 16 steps x
 * pace_gbs 5750, 6000, 6125, 6250, 6375, 6500 or 6750), each as back-to-back
 * launches, then the four fastest again with three times the launches,
 * on this request table with HIP events, check
 * that every candidate's output has the same checksum, keep the fastest as
 * the batch configuration, and report all of them. `out` receives the
 * requests' output. reps: timed launches per candidate (>= 1).
 * Errors: as rngx_generate_batch; RNGX_E_HIP if two candidates disagree. */
int rngx_autotune_batch(const rngx_req *reqs, uint32_t m, uint64_t *out, uint64_t out_cap,
                        uint32_t reps, void *stream, rngx_tune_result *result);

/* Autotuner of the plain generator's launch configuration (the batched
 * autotuner's counterpart, for rngx_generate / rngx_generate_u32): time
 * every configuration block {256, 512, 1024} x chunks {1, 2, 4} x
 * nontemporal {0, 1} (18 bases), then row schedules (pace_gbs): every
 * base at 6000, 6750 and 7500 GB/s, and the two bases fastest with a
 * schedule at 5500..8000 GB/s in steps of 250 (88 candidates in all),
 * then the four fastest again with three times the launches, on
 * the current generator (its n_states) for n_iters
 * iterations on `stream`, with HIP events around each candidate's timed
 * launches; every candidate starts from a snapshot of the states, so all
 * of them write the
 * same values, V(seed, g, cursor + k) for k < n_iters, which is checked by
 * checksum. The fastest becomes the launch configuration of that output type
 * (as rngx_set_launch would set it). On return `out` holds those values and
 * the generator's states and cursor are as before the call.
 * out: device memory of n_iters * n_states values (8-byte, or 4-byte with
 * u32, aligned). reps: launches per candidate, run back to back and timed
 * together (>= 1). The snapshot
 * (8 * n_states bytes) is allocated and freed by the call.
 * Errors: RNGX_E_NOINIT; RNGX_E_INVAL (NULL result or out, misaligned out,
 * reps or n_iters 0); RNGX_E_NOMEM; RNGX_E_HIP (also when two candidates
 * disagree). */
typedef struct rngx_plain_tune_entry {
    rngx_launch cfg;
    double ms; /* mean kernel time over the timed launches */
} rngx_plain_tune_entry;
typedef struct rngx_plain_tune_result {
    rngx_launch best;
    double best_ms;  /* the best confirmation timing */
    double best_gbs; /* algorithmic bytes (output + 16 per state) / best_ms */
    uint32_t n_tried;
    uint32_t reserved;
    rngx_plain_tune_entry tried[RNGX_TUNE_MAX];
    /* The RNGX_TUNE_CONFIRM fastest candidates timed again with 3 * reps
     * launches each (fewer if fewer were tried; unused entries zero); best
     * is the fastest of these. */
    rngx_plain_tune_entry confirm[RNGX_TUNE_CONFIRM];
} rngx_plain_tune_result;
int rngx_autotune_plain(uint32_t n_iters, int u32, void *out, uint32_t reps, void *stream,
                        rngx_plain_tune_result *result);

/* Tuning cache: the chosen launch configurations kept across processes, one
 * JSON object per line, keyed by device (architecture name and compute-unit
 * count) and kind ("plain_u64", "plain_u32", "batch"), with the shape it was
 * tuned on and its time.
 * rngx_tune_cache_save: write the current device's three configurations
 *   (rngx_get_launch for u64 and u32, rngx_get_batch_cfg) into `path`,
 *   replacing that device's earlier entries and keeping every other line.
 * rngx_tune_cache_load: apply the entries recorded for the current device
 *   (as rngx_set_launch / rngx_set_batch_cfg); *applied (may be NULL) gets
 *   their number. Entries of other devices are ignored.
 * With the environment variable RNGX_TUNE_CACHE naming a file, the first
 * successful rngx_init of the process loads it (if it exists), and each
 * autotuner (rngx_autotune_plain, rngx_autotune_batch) records its choice
 * there.
 * Errors: RNGX_E_INVAL (NULL path, a file that cannot be read or written, a
 * line that is not a tuning entry, an invalid configuration); RNGX_E_HIP. */
int rngx_tune_cache_save(const char *path);
int rngx_tune_cache_load(const char *path, uint32_t *applied);

/* Order-sensitive checksum sum_i data[i] * (2 i + 1) mod 2^64 of n device
 * values, computed on the device; waits for `stream` and writes *result.
 * Errors: RNGX_E_INVAL (NULL result, NULL data with n > 0); RNGX_E_HIP. */
int rngx_checksum(const uint64_t *data, uint64_t n, void *stream, uint64_t *result);

/* Host-side helpers of the same definitions (no GPU needed):
 * rngx_initial_state: *out = H(seed, gid) (Listing S4 with the seed folded in);
 * rngx_jump_ahead:    *out = XS^k(state), by GF(2) jump-ahead. */
int rngx_initial_state(uint64_t seed, uint32_t gid, uint64_t *out);
int rngx_jump_ahead(uint64_t state, uint64_t k, uint64_t *out);

/* ------------------------------------------------------------------------ */
/* Serving                                                                   */
/* ------------------------------------------------------------------------ */

/* Start the request server. It seeds n_states resident base states
 * H(seed, g) once (the init kernel) and keeps them on the device; each
 * stream g then has a cursor that starts at 0. Requests are admitted, in
 * submission order, as the output pool has room, grouped into launches of
 * the batched kernel (at most max_batch requests each), and run on up to
 * n_streams HIP streams at once, with up to two launches queued per stream:
 * requests arriving while others run are admitted and launched as soon as
 * memory and a launch slot are free.
 * pool: caller-owned device memory of pool_bytes bytes, 256-byte aligned,
 *       kept alive until rngx_serve_stop; results are written into it.
 * Batches are launched directly (no graph) with a schedule chosen by their
 * size, independent of the batch configuration: up to 2^23 values, one wave
 * per 1,024-value item (tables of up to 16 requests in the kernel's
 * arguments); larger, the persistent grid with 256 values per lane, at most
 * 8 waves per compute unit, fitted to the batch.
 * Errors: RNGX_E_BUSY if already running; RNGX_E_INVAL (n_states == 0, NULL
 * or misaligned pool, pool_bytes < 256, n_streams outside 1..16,
 * max_batch == 0); RNGX_E_NOMEM; RNGX_E_HIP. */
int rngx_serve_start(uint64_t seed, uint32_t n_states, void *pool, uint64_t pool_bytes,
                     uint32_t n_streams, uint32_t max_batch);

/* Free a request's pool memory as soon as it completes (results unread). */
#define RNGX_SERVE_AUTORELEASE 1u

/* Submit a request for the next `length` values of stream `stream_id`. The
 * values are reserved now: if c is the stream's cursor, the result is
 *     V(seed, stream_id, c + t),  t < length,
 * and the cursor becomes c + length. The result therefore does not depend on
 * what the request is batched with or when it runs. *ticket identifies it.
 * rngx_serve_submit waits while the pending bound (rngx_serve_set_max_pending)
 * is reached; rngx_serve_try_submit returns RNGX_E_BUSY instead.
 * Errors: RNGX_E_NOINIT (not running); RNGX_E_INVAL (NULL ticket, stream out
 * of range, length 0 or above the pool, unknown flags, a cursor that would
 * pass value number 2^64 - 1); RNGX_E_BUSY. */
int rngx_serve_submit(uint32_t stream_id, uint64_t length, uint32_t flags, uint64_t *ticket);
int rngx_serve_try_submit(uint32_t stream_id, uint64_t length, uint32_t flags,
                          uint64_t *ticket);

/* Submit k requests at once (one lock acquisition), in array order, with the
 * semantics of rngx_serve_submit; tickets (optional) receives their tickets.
 * On an error, the requests before the failing one have been submitted. */
int rngx_serve_submit_many(const uint32_t *stream_ids, const uint64_t *lengths, uint64_t k,
                           uint32_t flags, uint64_t *tickets);

/* State of a request: *done = 1 once its values are in the pool; *values is
 * their device address once the request is admitted (NULL before).
 * Errors: RNGX_E_NOINIT; RNGX_E_INVAL (unknown or released ticket). */
int rngx_serve_poll(uint64_t ticket, uint64_t **values, int *done);

/* Block until the request is done (or timeout_s passes: RNGX_E_BUSY). */
int rngx_serve_wait(uint64_t ticket, double timeout_s, uint64_t **values);

/* Give a done request's pool memory back (the consumer has read it).
 * Errors: RNGX_E_INVAL (unknown ticket); RNGX_E_BUSY (not done yet). */
int rngx_serve_release(uint64_t ticket);

/* Latency is measured from submission to the moment the server sees the
 * request's batch complete; queue wait from submission to admission. GB/s is
 * completed output bytes over the time from the first submission to the last
 * completion since the statistics were reset. */
typedef struct rngx_serve_report {
    uint64_t submitted, completed, released;
    uint64_t pending, admitted, inflight_batches;
    uint64_t batches, bytes;
    double elapsed_s, gbs;
    double lat_p50_us, lat_p99_us, lat_max_us, lat_mean_us;
    double wait_p50_us, wait_p99_us;     /* submission -> admission */
    double launch_p50_us, launch_p99_us; /* submission -> launch issued */
    double exec_p50_us, exec_p99_us;     /* launch issued -> completion seen */
    uint64_t max_pending, admission_stalls;
    double mean_batch_requests;
    uint64_t pool_bytes, pool_used_bytes, pool_peak_bytes;
    /* Requests of rngx_serve_run_trace only: submission lag, the time from a
     * request's scheduled arrival to its actual submission (their latency
     * above is measured from the scheduled arrival, so it includes this). */
    double lag_p50_us, lag_p99_us, lag_max_us;
} rngx_serve_report;

int rngx_serve_stats(rngx_serve_report *out);
int rngx_serve_reset_stats(void);

/* Open-loop load driver: submit request i (stream_id[i], length[i], with
 * RNGX_SERVE_AUTORELEASE) at arrival_s[i] seconds after the call starts
 * (arrival_s non-decreasing; the requests already due are submitted together,
 * by rngx_serve_submit_many in chunks of at most 512, so equal arrival times
 * form a backlog),
 * then wait until every request has completed
 * (at most timeout_s) and report the statistics of this trace (they are
 * reset at the start). A traced request's latency, admission wait and
 * launch delay are measured from its scheduled arrival, not from its actual
 * submission, so any lag of the submitting thread (for instance while the
 * scheduler holds the server's lock) counts against them; the lag itself is
 * reported as lag_*. Errors: as rngx_serve_submit; RNGX_E_BUSY on timeout. */
int rngx_serve_run_trace(const double *arrival_s, const uint32_t *stream_id,
                         const uint64_t *length, uint64_t k, double timeout_s,
                         rngx_serve_report *out);

/* Bound on pending (not yet admitted) requests: submit waits and try_submit
 * returns RNGX_E_BUSY beyond it (default 2^20; kept across restarts).
 * Errors: RNGX_E_INVAL if max_pending == 0. */
int rngx_serve_set_max_pending(uint64_t max_pending);

/* Bound on batches in flight (launched and not yet complete; default 2, kept
 * across restarts). While that many run, newly admitted requests wait and
 * join the next batch: under load batches grow instead of many small ones
 * competing on the device, and one batch stays queued behind the running
 * one. A batch of at most 2^20 values, which is latency-bound, may run one
 * above the bound. Errors: RNGX_E_INVAL unless 1 <= max_inflight <= 32. */
int rngx_serve_set_max_inflight(uint32_t max_inflight);

/* Stop the server: requests not yet launched are dropped, launched batches
 * are waited for, resident states and streams are freed (the pool is the
 * caller's). Safe to call when not running. */
int rngx_serve_stop(void);

/* ------------------------------------------------------------------------ */
/* Event profiling (the profiler module, Section 4.3; summary of Fig. 3)     */
/* ------------------------------------------------------------------------ */

#define RNGX_PROF_NAME 32
#define RNGX_PROF_MAX_AGG 16
#define RNGX_PROF_MAX_OVERLAP 32

/* One timed operation: its name (INIT_KERNEL, RNG_KERNEL, READ_BUFFER, ...),
 * an id of the stream (queue) it ran on, and its start and end instants in
 * nanoseconds from the start of the profiling window. */
typedef struct rngx_prof_event {
    char name[RNGX_PROF_NAME];
    uint64_t queue;
    uint64_t start_ns;
    uint64_t end_ns;
} rngx_prof_event;

typedef struct rngx_prof_agg {
    char name[RNGX_PROF_NAME];
    uint64_t count;
    double abs_s;   /* sum of durations of the events of this name */
    double rel_pct; /* abs_s as a share of the sum over all events */
} rngx_prof_agg;

typedef struct rngx_prof_overlap {
    char name1[RNGX_PROF_NAME];
    char name2[RNGX_PROF_NAME];
    double overlap_s; /* summed intersection of events of the two names */
} rngx_prof_overlap;

/* Profile analysis. Aggregates are sorted by time, descending; overlap rows
 * by duration, descending. Two events overlap only if they ran on different
 * queues; an overlap row is an unordered pair of names, printed with the
 * name of smaller aggregate time first. eff_s = total_s - overlap_s
 * ("Tot. of all events (eff.)"), device_pct = 100 * eff_s / elapsed_s. */
typedef struct rngx_prof_stats {
    uint64_t n_events;
    uint64_t n_dropped; /* events not logged because the log was full */
    uint32_t n_agg;
    uint32_t n_overlap;
    double total_s;
    double overlap_s;
    double eff_s;
    double elapsed_s; /* host wall clock of the profiling window */
    double device_pct;
    double host_pct;
    rngx_prof_agg agg[RNGX_PROF_MAX_AGG];
    rngx_prof_overlap overlap[RNGX_PROF_MAX_OVERLAP];
} rngx_prof_stats;

/* Clear the event log and open a new profiling window (host clock starts).
 * Errors: RNGX_E_NOINIT before rngx_init. */
int rngx_profile_start(void);

/* The same as rngx_profile_start: the log restarts empty (the name used for
 * the operation in the library's call list). */
int rngx_profile_reset(void);

/* Wait for every logged operation to finish and close the window. */
int rngx_profile_stop(void);

/* Turn event logging on (default) or off. */
int rngx_profile_enable(int on);

/* Summary text in the layout of Fig. 3 for the current window (closing it
 * first if it is open). The text is owned by the library and stays valid
 * until the next call of rngx_profile. Returns NULL on error. */
const char *rngx_profile(void);

/* The same analysis as structured data. */
int rngx_profile_stats(rngx_prof_stats *out);

/* Copy up to cap logged events (closing the window first if it is open);
 * *n_out receives the number of logged events. */
int rngx_profile_events(rngx_prof_event *out, uint32_t cap, uint32_t *n_out);

/* Analyse a caller-supplied event table (host memory) with the same code.
 * Errors: RNGX_E_INVAL if any event ends before it starts, or events is
 * NULL with n > 0. */
int rngx_profile_analyze(const rngx_prof_event *events, uint32_t n,
                         double elapsed_s, rngx_prof_stats *out);

/* Export formats of an event table (Section 4.3: the profiler can write a
 * table of queue name, start instant, end instant and event name to a text
 * file for a queue-utilisation chart, as in Fig. 5).
 * RNGX_EXPORT_TABLE: tab-separated text, a header line
 *   "queue<TAB>t_start<TAB>t_end<TAB>event", then one line per event in order
 *   of start time (ties: table order); instants in ns; queues are named
 *   q0, q1, ... in order of their first event.
 * RNGX_EXPORT_TRACE: Chrome trace-event JSON (one complete event per event,
 *   one track per queue named as above, times in microseconds), which
 *   Perfetto and chrome://tracing open. */
#define RNGX_EXPORT_TABLE 0
#define RNGX_EXPORT_TRACE 1

/* Write a caller-supplied event table (host memory) to the file at `path`
 * (created or truncated). Errors: RNGX_E_INVAL (path NULL, events NULL with
 * n > 0, an event that ends before it starts, an unknown format, or the file
 * cannot be written; rngx_last_error names the cause). */
int rngx_profile_write(const rngx_prof_event *events, uint32_t n, const char *path, int format);

/* Write the current window's event table (closing the window first if it is
 * open). Errors: RNGX_E_NOINIT if no window was ever opened; otherwise as
 * rngx_profile_write. */
int rngx_profile_export(const char *path, int format);

#ifdef __cplusplus
}
#endif

#endif /* RNGX_H */
