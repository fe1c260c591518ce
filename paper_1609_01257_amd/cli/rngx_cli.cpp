// rngx_cli: the generator as a command-line program with the interface of the
// paper's example (Section 5): given n (values per iteration) and i
// (iterations) it writes the 8 * n * i bytes of raw 64-bit values to
// standard output, iteration after iteration, work-item g at position g
// within an iteration, in host byte order. With seed 0 the byte stream is the
// one the paper's program writes: iteration 0 is the initial states, and
// each later iteration is one xorshift step of the previous one.
//
// Generation and device-to-host copies are overlapped on two streams by
// rngx_stream_to_host; the host writes each step out while the device works
// on the next ones (host_slots page-locked slots).
//
// Usage: rngx_cli [-s seed] [-u] [-x] [-k iters_per_step] [-h host_slots] n i
//   -s seed   64-bit seed (decimal or 0x hex), default 0;
//   -u        write 32-bit values (4 * n * i bytes);
//   -x        the scrambled variant (each value times 2685821657736338717
//             modulo 2^64, the high half with -u) instead of the states;
//   -k        iterations per generation launch and copy, default 1;
//   -h        host slots, default 2.
// Exit status 0 on success, 1 on a library or I/O error (message on stderr),
// 2 on a usage error.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "rngx.h"

namespace {

int consume(void *user, uint64_t, const void *values, size_t bytes)
{
    return std::fwrite(values, 1, bytes, static_cast<FILE *>(user)) == bytes ? 0 : 1;
}

int usage(const char *msg)
{
    std::fprintf(stderr, "rngx_cli: %s\nusage: rngx_cli [-s seed] [-u] [-x] [-k iters_per_step] "
                         "[-h host_slots] n i\n", msg);
    return 2;
}

bool parse_u64(const char *s, unsigned long long max, unsigned long long *v)
{
    if (!s || !*s || *s == '-')
        return false;
    char *end = nullptr;
    errno = 0;
    const unsigned long long x = std::strtoull(s, &end, 0);
    if (errno || *end || x > max)
        return false;
    *v = x;
    return true;
}

int fail(const char *what, int rc)
{
    std::fprintf(stderr, "rngx_cli: %s: %s: %s\n", what, rngx_strerror(rc), rngx_last_error());
    return 1;
}

} // namespace

int main(int argc, char **argv)
{
    unsigned long long seed = 0, k = 1, slots = 2, n = 0, iters = 0;
    int u32 = 0, star = 0, pos = 0;
    const char *args[2] = {nullptr, nullptr};
    for (int a = 1; a < argc; ++a) {
        if (!std::strcmp(argv[a], "-u")) {
            u32 = 1;
        } else if (!std::strcmp(argv[a], "-x")) {
            star = 1;
        } else if (!std::strcmp(argv[a], "-s") || !std::strcmp(argv[a], "-k") ||
                   !std::strcmp(argv[a], "-h")) {
            if (a + 1 >= argc)
                return usage("missing option value");
            const char opt = argv[a][1];
            unsigned long long *dst = opt == 's' ? &seed : opt == 'k' ? &k : &slots;
            const unsigned long long max = opt == 's' ? ~0ull : 0xffffffffull;
            if (!parse_u64(argv[++a], max, dst) || (opt != 's' && *dst == 0))
                return usage("bad option value");
        } else if (pos < 2) {
            args[pos++] = argv[a];
        } else {
            return usage("too many arguments");
        }
    }
    if (pos != 2 || !parse_u64(args[0], 0xffffffffull, &n) || n == 0 ||
        !parse_u64(args[1], 0xffffffffull, &iters))
        return usage("need n (1..2^32-1) and i (0..2^32-1)");
    if (k > iters && iters > 0)
        k = iters;
    const size_t esize = u32 ? 4 : 8;
    // Two device buffers and `slots` host slots of one step each.
    if (k > (1ull << 40) / (n * esize) / slots)
        return usage("a step of k iterations times host slots exceeds 1 TiB");
    const size_t step_bytes = (size_t)k * n * esize;

    int rc = rngx_set_scrambler(star ? RNGX_SCRAMBLE_STAR : RNGX_SCRAMBLE_NONE);
    if (rc)
        return fail("rngx_set_scrambler", rc);
    rc = rngx_init(seed, (uint32_t)n);
    if (rc)
        return fail("rngx_init", rc);
    void *dev[2] = {nullptr, nullptr}, *host = nullptr;
    int status = 0;
    if (hipMalloc(&dev[0], step_bytes) != hipSuccess || hipMalloc(&dev[1], step_bytes) != hipSuccess ||
        hipHostMalloc(&host, step_bytes * slots, hipHostMallocDefault) != hipSuccess) {
        std::fprintf(stderr, "rngx_cli: cannot allocate %zu-byte step buffers\n", step_bytes);
        status = 1;
    }
    // Whole steps of k iterations, then one step with the remainder.
    const unsigned long long full = k ? iters / k : 0, rest = k ? iters % k : 0;
    if (!status && full) {
        rc = rngx_stream_to_host((uint32_t)full, (uint32_t)k, u32, dev[0], dev[1], step_bytes,
                                 host, (uint32_t)slots, consume, stdout, nullptr, nullptr);
        if (rc)
            status = fail("rngx_stream_to_host", rc);
    }
    if (!status && rest) {
        rc = rngx_stream_to_host(1, (uint32_t)rest, u32, dev[0], dev[1], step_bytes, host,
                                 (uint32_t)slots, consume, stdout, nullptr, nullptr);
        if (rc)
            status = fail("rngx_stream_to_host", rc);
    }
    if (std::fflush(stdout) != 0 && !status) {
        std::fprintf(stderr, "rngx_cli: write error: %s\n", std::strerror(errno));
        status = 1;
    }
    if (host)
        (void)hipHostFree(host);
    for (void *d : dev)
        if (d)
            (void)hipFree(d);
    rc = rngx_shutdown();
    if (rc && !status)
        status = fail("rngx_shutdown", rc);
    return status;
}
