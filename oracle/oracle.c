/*
 * oracle.c -- plain, sequential CPU definition of the massive pseudo-random
 * number generator in the example application of "cf4ocl: a C framework for
 * OpenCL" (Section 5, "Example: massive pseudo-random number generator";
 * supplementary Listing S4, the init kernel, and Listing S5, the rng kernel).
 *
 * TEST INFRASTRUCTURE. This file is the checker, not the product: only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. The GPU library (paper_1609_01257_amd) never links, loads or calls it,
 * and the two share no source, header, table or constant.
 *
 * Arithmetic: unsigned integers only. 32-bit words wrap modulo 2^32, 64-bit
 * words wrap modulo 2^64, right shifts are logical. Everything is computed
 * one work-item at a time and one step at a time; there is no jump-ahead, no
 * blocking and no reordering, so each function can be read against the paper
 * line by line.
 *
 * Readings of the paper that this file fixes (the paper is silent on them):
 *  - Seed. The paper's init kernel hashes only the global index. A 64-bit
 *    seed s is folded in so that s = 0 gives exactly the paper's states (see
 *    oracle_init_state).
 *  - Emission order. The values written by init are the first batch of
 *    output (Section 5), so iteration k of a stream emits the state after k
 *    xorshift steps: emit first, then advance.
 *  - Word order. Init stores the low hash in the .x half and the high hash in
 *    the .y half of a uint2 that the rng kernel then reads as one ulong, i.e.
 *    the state is (high << 32) | low on a little-endian device.
 *
 * The scrambled variant (oracle_scramble, oracle_generate_star*) follows
 * the paper's remark that a more complex generator would cost nothing; its
 * reading (the xorshift* output multiplication) is stated where it is
 * defined, and it is pinned by linear complexity, the odd multiplier's
 * inverse and the shared state sequence.
 *
 * Pins: the oracle's own tests check it against hand-traced values, the
 * full-period property of the (21,35,4) xorshift over GF(2), bijectivity of
 * both 32-bit hashes, the never-zero invariant, concatenation and transpose
 * identities, and bit-frequency sanity. The seeded extension for s != 0 has
 * no counterpart in the paper: its values are pinned only by its written
 * definition and those invariants (parity against the paper unpinned by
 * construction for s != 0).
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>

/* ------------------------------------------------------------------------- */
/* Listing S4, "low bits": the six-round 32-bit integer hash (Bob Jenkins'     */
/* mix, as cited in the kernel's comment). Input: the work-item's global      */
/* index truncated to 32 bits.                                                */
/* ------------------------------------------------------------------------- */
uint32_t oracle_hash_low(uint32_t a)
{
    a = (a + 0x7ed55d16u) + (a << 12);
    a = (a ^ 0xc761c23cu) ^ (a >> 19);
    a = (a + 0x165667b1u) + (a << 5);
    a = (a + 0xd3a2646cu) ^ (a << 9);
    a = (a + 0xfd7046c5u) + (a << 3);
    a = (a ^ 0xb55a4f09u) ^ (a >> 16);
    return a;
}

/* ------------------------------------------------------------------------- */
/* Listing S4, "high bits": the five-round shift-multiply hash (Thomas Wang's */
/* integer hash, cited by Section 5). Input: the low word.                    */
/* ------------------------------------------------------------------------- */
uint32_t oracle_hash_high(uint32_t a)
{
    a = (a ^ 61u) ^ (a >> 16);
    a = a + (a << 3);
    a = a ^ (a >> 4);
    a = a * 0x27d4eb2du;
    a = a ^ (a >> 15);
    return a;
}

/* ------------------------------------------------------------------------- */
/* Initial state of work-item gid (Listing S4; Section 5: the init kernel     */
/* hashes the global ID and its output is both the first batch of numbers and */
/* the seed of the next batch).                                               */
/*                                                                            */
/* Paper (seed 0): low = J(gid), high = W(low), state = high:low.             */
/* Seeded reading (not in the paper):                                         */
/*   l = J(lo32 seed) ^ J(0),  h = W(hi32 seed) ^ W(0)                        */
/*   low = J(gid ^ l),         high = W(low ^ h)                              */
/* At seed 0, l = h = 0 and this is exactly the paper. The all-zero state is  */
/* the xorshift's fixed point; if it ever arises it is replaced by W(0)<<32.  */
/* At seed 0 it cannot arise, because high = W(low) and W(0) != 0.            */
/* ------------------------------------------------------------------------- */
uint64_t oracle_init_state(uint64_t seed, uint32_t gid)
{
    uint32_t l = oracle_hash_low((uint32_t)(seed & 0xffffffffu)) ^ oracle_hash_low(0u);
    uint32_t h = oracle_hash_high((uint32_t)(seed >> 32)) ^ oracle_hash_high(0u);
    uint32_t low = oracle_hash_low(gid ^ l);
    uint32_t high = oracle_hash_high(low ^ h);
    uint64_t state = ((uint64_t)high << 32) | (uint64_t)low;
    if (state == 0u)
        state = (uint64_t)oracle_hash_high(0u) << 32;
    return state;
}

/* ------------------------------------------------------------------------- */
/* Listing S5: one step of Marsaglia's 64-bit xorshift with shifts (21,35,4): */
/* left 21, right 35, left 4, each xor-ed into the state in that order.       */
/* ------------------------------------------------------------------------- */
uint64_t oracle_rng_step(uint64_t x)
{
    x ^= x << 21;
    x ^= x >> 35;
    x ^= x << 4;
    return x;
}

/* Value number k of the stream of work-item gid: k sequential steps from the
 * initial state (Section 5: each invocation of the rng kernel advances every
 * state once). */
uint64_t oracle_value(uint64_t seed, uint32_t gid, uint64_t k)
{
    uint64_t x = oracle_init_state(seed, gid);
    for (uint64_t t = 0; t < k; ++t)
        x = oracle_rng_step(x);
    return x;
}

/* ------------------------------------------------------------------------- */
/* Plain output (Eq. 1: n values per iteration, i iterations, 8*n*i bytes).   */
/* After the generator has been seeded for n work-items and has already       */
/* produced `cursor` iterations, the next n_iters iterations are              */
/*     out[k*n + g] = value(seed, g, cursor + k),  k < n_iters, g < n,        */
/* iteration-major, which is the byte order the paper's program writes to     */
/* its standard output. The loops follow the paper's program: one array of   */
/* n states; each iteration emits every state, then advances every state one  */
/* step (Section 5). Returns the number of zero values produced (the          */
/* never-zero invariant says it is always 0), or UINT64_MAX if the state      */
/* array cannot be allocated.                                                 */
/* ------------------------------------------------------------------------- */
static uint64_t *seeded_states(uint64_t seed, uint32_t n, uint64_t cursor)
{
    uint64_t *st = (uint64_t *)malloc((size_t)n * sizeof(uint64_t) + 1);
    if (!st)
        return NULL;
    for (uint32_t g = 0; g < n; ++g)
        st[g] = oracle_value(seed, g, cursor);
    return st;
}

uint64_t oracle_generate(uint64_t seed, uint32_t n, uint64_t cursor,
                         uint32_t n_iters, uint64_t *out)
{
    uint64_t zeros = 0;
    uint64_t *st = seeded_states(seed, n, cursor);
    if (!st)
        return UINT64_MAX;
    for (uint32_t k = 0; k < n_iters; ++k) {
        for (uint32_t g = 0; g < n; ++g) {
            if (st[g] == 0u)
                ++zeros;
            out[(size_t)k * n + g] = st[g];
            st[g] = oracle_rng_step(st[g]);
        }
    }
    free(st);
    return zeros;
}

/* 32-bit form of the plain output: the low half of each 64-bit value. */
uint64_t oracle_generate_u32(uint64_t seed, uint32_t n, uint64_t cursor,
                             uint32_t n_iters, uint32_t *out)
{
    uint64_t zeros = 0;
    uint64_t *st = seeded_states(seed, n, cursor);
    if (!st)
        return UINT64_MAX;
    for (uint32_t k = 0; k < n_iters; ++k) {
        for (uint32_t g = 0; g < n; ++g) {
            if (st[g] == 0u)
                ++zeros;
            out[(size_t)k * n + g] = (uint32_t)(st[g] & 0xffffffffu);
            st[g] = oracle_rng_step(st[g]);
        }
    }
    free(st);
    return zeros;
}

/* ------------------------------------------------------------------------- */
/* Scrambled output variant. The paper observes (discussing the queue chart   */
/* of Fig. 5) that its generator kernels are much shorter than the transfers, */
/* so a more complex generator would cost nothing and give better numbers.    */
/* Reading: the xorshift* construction (S. Vigna, "An experimental           */
/* exploration of Marsaglia's xorshift generators, scrambled", ACM TOMS      */
/* 2016) applied to this generator. The state sequence is unchanged (same     */
/* seeding, same (21,35,4) steps, same cursor); only the emitted word        */
/* changes: the state times the odd constant 2685821657736338717 (that       */
/* paper's multiplier) modulo 2^64. An odd multiplier is a bijection of the  */
/* 64-bit words, so periods and the never-zero property carry over, while    */
/* the output bits stop being GF(2)-linear functions of the state. The       */
/* 32-bit form keeps the high half of the product, as that paper advises    */
/* (the low half of a product only depends on the low halves).               */
/* ------------------------------------------------------------------------- */
uint64_t oracle_scramble(uint64_t x)
{
    return x * 2685821657736338717ull;
}

/* The scrambled words of n given values (for the batched and served forms:
 * their scrambled output is the scrambled plain output, value by value). */
void oracle_scramble_n(const uint64_t *in, uint64_t n, uint64_t *out)
{
    for (uint64_t i = 0; i < n; ++i)
        out[i] = oracle_scramble(in[i]);
}

uint64_t oracle_generate_star(uint64_t seed, uint32_t n, uint64_t cursor,
                              uint32_t n_iters, uint64_t *out)
{
    uint64_t zeros = 0;
    uint64_t *st = seeded_states(seed, n, cursor);
    if (!st)
        return UINT64_MAX;
    for (uint32_t k = 0; k < n_iters; ++k) {
        for (uint32_t g = 0; g < n; ++g) {
            const uint64_t v = oracle_scramble(st[g]);
            if (v == 0u)
                ++zeros;
            out[(size_t)k * n + g] = v;
            st[g] = oracle_rng_step(st[g]);
        }
    }
    free(st);
    return zeros;
}

uint64_t oracle_generate_star_u32(uint64_t seed, uint32_t n, uint64_t cursor,
                                  uint32_t n_iters, uint32_t *out)
{
    uint64_t zeros = 0;
    uint64_t *st = seeded_states(seed, n, cursor);
    if (!st)
        return UINT64_MAX;
    for (uint32_t k = 0; k < n_iters; ++k) {
        for (uint32_t g = 0; g < n; ++g) {
            if (st[g] == 0u)
                ++zeros;
            out[(size_t)k * n + g] = (uint32_t)(oracle_scramble(st[g]) >> 32);
            st[g] = oracle_rng_step(st[g]);
        }
    }
    free(st);
    return zeros;
}

/* ------------------------------------------------------------------------- */
/* The same output, a slice at a time: the pieces a checker needs to compare  */
/* a very large output (gigabytes of rows) with the definition without        */
/* holding all of it, and to spread the work over host threads by work-item. */
/* Nothing here jumps ahead: every state is reached by sequential steps.      */
/* ------------------------------------------------------------------------- */

/* States of work-items g0 .. g0 + count - 1 (wrapping is not allowed: the    */
/* caller keeps g0 + count <= 2^32) at value number `cursor`, each one        */
/* stepped `cursor` times from its initial state (Listing S4, then Listing S5 */
/* once per earlier iteration).                                               */
void oracle_seed_range(uint64_t seed, uint32_t g0, uint64_t count, uint64_t cursor,
                       uint64_t *st)
{
    for (uint64_t t = 0; t < count; ++t)
        st[t] = oracle_value(seed, (uint32_t)(g0 + t), cursor);
}

/* Continue the paper's loop from a caller-held state array: n_rows more      */
/* iterations over `count` work-items. Iteration k emits every state into     */
/* row k (out[k * ld + t]), then advances every state one step (Section 5:    */
/* emit, then advance). On return st holds the next value of every stream,   */
/* so a second call continues exactly where the first stopped. `word`        */
/* selects the emitted word: 0 the state, 1 its low 32 bits (into a uint32   */
/* row), 2 the scrambled word, 3 the high half of the scrambled word (u32).  */
/* Returns the number of zero states met (never-zero invariant: always 0).   */
uint64_t oracle_emit_rows(uint64_t *st, uint64_t count, uint32_t n_rows, int word, void *out,
                          uint64_t ld)
{
    uint64_t zeros = 0;
    uint64_t *o64 = (uint64_t *)out;
    uint32_t *o32 = (uint32_t *)out;
    for (uint32_t k = 0; k < n_rows; ++k) {
        for (uint64_t t = 0; t < count; ++t) {
            const uint64_t x = st[t];
            if (x == 0u)
                ++zeros;
            const size_t at = (size_t)k * ld + t;
            switch (word) {
            case 1: o32[at] = (uint32_t)(x & 0xffffffffu); break;
            case 2: o64[at] = oracle_scramble(x); break;
            case 3: o32[at] = (uint32_t)(oracle_scramble(x) >> 32); break;
            default: o64[at] = x; break;
            }
            st[t] = oracle_rng_step(x);
        }
    }
    return zeros;
}

/* Plain output restricted to work-items g0 <= g < g1 (g1 <= 2^32):           */
/*     out[k * (g1 - g0) + (g - g0)] = value(seed, g, cursor + k),            */
/* i.e. the matching columns of oracle_generate. Returns the zero count, or  */
/* UINT64_MAX if the state array cannot be allocated.                        */
uint64_t oracle_generate_range(uint64_t seed, uint64_t g0, uint64_t g1, uint64_t cursor,
                               uint32_t n_iters, uint64_t *out)
{
    const uint64_t count = g1 > g0 ? g1 - g0 : 0;
    uint64_t *st = (uint64_t *)malloc((size_t)count * sizeof(uint64_t) + 1);
    if (!st)
        return UINT64_MAX;
    oracle_seed_range(seed, (uint32_t)g0, count, cursor, st);
    const uint64_t zeros = oracle_emit_rows(st, count, n_iters, 0, out, count);
    free(st);
    return zeros;
}

/* ------------------------------------------------------------------------- */
/* Batched streams. Request j names one stream by (seed_j, gid_j) and asks    */
/* for length_j consecutive values starting at value number offset_j. The     */
/* outputs are packed one request after another, in request order:           */
/*     out[base_j + t] = value(seed_j, gid_j, offset_j + t),  t < length_j,   */
/*     base_j = length_0 + ... + length_{j-1}.                                */
/* The oracle's request record is its own; it is laid out like the library's */
/* so the tests can pass one packed array to both.                            */
/* ------------------------------------------------------------------------- */
typedef struct oracle_req {
    uint64_t seed;
    uint64_t offset;
    uint64_t length;
    uint32_t gid;
    uint32_t reserved;
} oracle_req;

uint64_t oracle_generate_batch(const oracle_req *reqs, uint32_t m, uint64_t *out)
{
    uint64_t zeros = 0;
    size_t base = 0;
    for (uint32_t j = 0; j < m; ++j) {
        uint64_t x = oracle_value(reqs[j].seed, reqs[j].gid, reqs[j].offset);
        for (uint64_t t = 0; t < reqs[j].length; ++t) {
            if (x == 0u)
                ++zeros;
            out[base + t] = x;
            x = oracle_rng_step(x);
        }
        base += (size_t)reqs[j].length;
    }
    return zeros;
}

/* Bulk evaluation of the two hashes over consecutive inputs
 * start, start+1, ... (wrapping mod 2^32); used by the exhaustive tests. */
void oracle_hash_low_range(uint32_t start, uint64_t count, uint32_t *out)
{
    for (uint64_t t = 0; t < count; ++t)
        out[t] = oracle_hash_low((uint32_t)(start + t));
}

void oracle_hash_high_range(uint32_t start, uint64_t count, uint32_t *out)
{
    for (uint64_t t = 0; t < count; ++t)
        out[t] = oracle_hash_high((uint32_t)(start + t));
}
