/* Exercises every function of oracle.c once, including edge sizes, in a
 * build with address and undefined-behaviour sanitizers (the test links this
 * file with oracle.c). Prints "ok" when the cross-checks below hold. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct oracle_req {
    uint64_t seed, offset, length;
    uint32_t gid, reserved;
} oracle_req;

uint32_t oracle_hash_low(uint32_t a);
uint32_t oracle_hash_high(uint32_t a);
uint64_t oracle_init_state(uint64_t seed, uint32_t gid);
uint64_t oracle_rng_step(uint64_t x);
uint64_t oracle_value(uint64_t seed, uint32_t gid, uint64_t k);
uint64_t oracle_generate(uint64_t seed, uint32_t n, uint64_t cursor, uint32_t n_iters,
                         uint64_t *out);
uint64_t oracle_generate_u32(uint64_t seed, uint32_t n, uint64_t cursor, uint32_t n_iters,
                             uint32_t *out);
uint64_t oracle_scramble(uint64_t x);
void oracle_scramble_n(const uint64_t *in, uint64_t n, uint64_t *out);
uint64_t oracle_generate_star(uint64_t seed, uint32_t n, uint64_t cursor, uint32_t n_iters,
                              uint64_t *out);
uint64_t oracle_generate_star_u32(uint64_t seed, uint32_t n, uint64_t cursor, uint32_t n_iters,
                                  uint32_t *out);
uint64_t oracle_generate_batch(const oracle_req *reqs, uint32_t m, uint64_t *out);
void oracle_hash_low_range(uint32_t start, uint64_t count, uint32_t *out);
void oracle_hash_high_range(uint32_t start, uint64_t count, uint32_t *out);

#define CHECK(c)                                                                            \
    do {                                                                                    \
        if (!(c)) {                                                                         \
            printf("failed: %s (line %d)\n", #c, __LINE__);                                 \
            return 1;                                                                       \
        }                                                                                   \
    } while (0)

int main(void)
{
    const uint32_t n = 37, it = 5;
    uint64_t *a = malloc(sizeof(uint64_t) * n * it), *b = malloc(sizeof(uint64_t) * n * it);
    uint32_t *a32 = malloc(sizeof(uint32_t) * n * it);
    CHECK(a && b && a32);
    CHECK(oracle_generate(7, n, 3, it, a) == 0);
    for (uint32_t k = 0; k < it; ++k)
        for (uint32_t g = 0; g < n; ++g)
            CHECK(a[k * n + g] == oracle_value(7, g, 3 + k));
    CHECK(oracle_generate_u32(7, n, 3, it, a32) == 0);
    CHECK(a32[n + 1] == (uint32_t)a[n + 1]);
    CHECK(oracle_generate_star(7, n, 3, it, b) == 0);
    oracle_scramble_n(a, (uint64_t)n * it, a);
    for (uint32_t i = 0; i < n * it; ++i)
        CHECK(a[i] == b[i]);
    CHECK(oracle_generate_star_u32(7, n, 3, it, a32) == 0);
    CHECK(a32[2] == (uint32_t)(b[2] >> 32));
    CHECK(oracle_generate(0, 1, 0, 0, a) == 0); /* zero iterations */

    oracle_req reqs[3] = {{1, 0, 4, 0, 0}, {2, 9, 0, 5, 0}, {3, 100, 2, 6, 0}};
    uint64_t out[6];
    CHECK(oracle_generate_batch(reqs, 3, out) == 0);
    CHECK(out[0] == oracle_init_state(1, 0) && out[4] == oracle_value(3, 6, 100));
    CHECK(oracle_rng_step(out[4]) == out[5]);

    uint32_t lo[8], hi[8];
    oracle_hash_low_range(0xfffffffcu, 8, lo); /* wraps past 2^32 - 1 */
    oracle_hash_high_range(0xfffffffcu, 8, hi);
    for (uint32_t i = 0; i < 8; ++i) {
        CHECK(lo[i] == oracle_hash_low(0xfffffffcu + i));
        CHECK(hi[i] == oracle_hash_high(0xfffffffcu + i));
    }
    CHECK(oracle_scramble(1) == 2685821657736338717ull);
    free(a);
    free(b);
    free(a32);
    printf("ok\n");
    return 0;
}
