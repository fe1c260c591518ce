/* Exhaustive bijectivity scan of a 32-bit function (test helper).
 * The function is supplied as a bulk evaluator range(start, count, out) that
 * fills out[t] = f(start + t). Every output is marked in a shared 512 MiB
 * bitmap with an atomic or; the return value counts outputs that were
 * already marked, so it is 0 iff f is a bijection on 32-bit words. */
#include <stdint.h>
#include <stdlib.h>

typedef void (*range_fn)(uint32_t start, uint64_t count, uint32_t *out);

int64_t count_collisions(range_fn f)
{
    const uint64_t chunk = (uint64_t)1 << 20;
    const int64_t nchunks = (int64_t)(((uint64_t)1 << 32) / chunk);
    uint64_t *bits = calloc((size_t)1 << 26, sizeof(uint64_t));
    if (!bits)
        return -1;
    int64_t dup = 0;
#pragma omp parallel reduction(+ : dup)
    {
        uint32_t *buf = malloc(chunk * sizeof(uint32_t));
#pragma omp for schedule(static)
        for (int64_t c = 0; c < nchunks; ++c) {
            f((uint32_t)(c * chunk), chunk, buf);
            for (uint64_t t = 0; t < chunk; ++t) {
                uint32_t y = buf[t];
                uint64_t b = (uint64_t)1 << (y & 63);
                uint64_t old = __atomic_fetch_or(&bits[y >> 6], b, __ATOMIC_RELAXED);
                if (old & b)
                    ++dup;
            }
        }
        free(buf);
    }
    free(bits);
    return dup;
}
