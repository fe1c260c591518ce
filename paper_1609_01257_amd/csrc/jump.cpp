// GF(2) jump-ahead for the (21,35,4) xorshift.
//
// Every xorshift step is linear over GF(2): x -> T x for a 64 x 64 bit
// matrix T (Listing S5's three shift-xors). Advancing a state by k steps is
// T^k x = prod over the set bits b of k of T^(2^b) applied to x, so a stream
// can start anywhere without stepping through its prefix (the F2-linear
// jump-ahead idea of Haramoto et al., 2008). The paper notes that xorshift
// is awkward to partition across parallel work; these tables are what lets
// one long stream be split into independent chunks here.
//
// Matrix layout: row r of a matrix is a uint64 whose bit j says whether
// output bit r depends on input bit j, so (M x)_r = parity(row_r & x). The
// GPU kernels keep row r in lane r and form M x with one ballot.
#include <cstring>
#include <mutex>

#include "internal.h"

namespace rngx {
namespace {

struct Tables {
    uint64_t pow2[64][64]; // pow2[b] = T^(2^b)
    bool ready = false;
};

Tables &tables()
{
    static Tables *t = new Tables;
    return *t;
}

std::mutex g_tables_mu;

uint64_t matvec(const uint64_t *m, uint64_t x)
{
    uint64_t y = 0;
    for (int r = 0; r < 64; ++r)
        y |= (uint64_t)(__builtin_popcountll(m[r] & x) & 1) << r;
    return y;
}

// c = a * b (apply b first, then a): row r of c = XOR of rows j of b over the
// set bits j of row r of a.
void matmul(const uint64_t *a, const uint64_t *b, uint64_t *c)
{
    uint64_t out[64];
    for (int r = 0; r < 64; ++r) {
        uint64_t acc = 0, row = a[r];
        while (row) {
            const int j = __builtin_ctzll(row);
            acc ^= b[j];
            row &= row - 1;
        }
        out[r] = acc;
    }
    std::memcpy(c, out, sizeof out);
}

} // namespace

const uint64_t *jump_tables()
{
    std::lock_guard<std::mutex> lk(g_tables_mu);
    Tables &t = tables();
    if (!t.ready) {
        // Column j of T is the step applied to the unit vector e_j.
        uint64_t rows[64] = {0};
        for (int j = 0; j < 64; ++j) {
            const uint64_t col = xs_step((uint64_t)1 << j);
            for (int r = 0; r < 64; ++r)
                rows[r] |= ((col >> r) & 1u) << j;
        }
        std::memcpy(t.pow2[0], rows, sizeof rows);
        for (int b = 1; b < 64; ++b)
            matmul(t.pow2[b - 1], t.pow2[b - 1], t.pow2[b]);
        t.ready = true;
    }
    return &t.pow2[0][0];
}

uint64_t jump_host(uint64_t x, uint64_t k)
{
    const uint64_t *pow2 = jump_tables();
    while (k) {
        const int b = __builtin_ctzll(k);
        x = matvec(pow2 + 64 * b, x);
        k &= k - 1;
    }
    return x;
}

void power_rows(uint64_t k, uint64_t *rows_out)
{
    const uint64_t *pow2 = jump_tables();
    uint64_t acc[64];
    for (int r = 0; r < 64; ++r)
        acc[r] = (uint64_t)1 << r;
    while (k) {
        const int b = __builtin_ctzll(k);
        matmul(pow2 + 64 * b, acc, acc); // powers of T commute
        k &= k - 1;
    }
    std::memcpy(rows_out, acc, sizeof acc);
}

} // namespace rngx

extern "C" int rngx_jump_ahead(uint64_t state, uint64_t k, uint64_t *out)
{
    rngx::clear_error();
    if (!out)
        return rngx::set_error(RNGX_E_INVAL, "rngx_jump_ahead: out is NULL");
    *out = rngx::jump_host(state, k);
    return RNGX_OK;
}

extern "C" int rngx_initial_state(uint64_t seed, uint32_t gid, uint64_t *out)
{
    rngx::clear_error();
    if (!out)
        return rngx::set_error(RNGX_E_INVAL, "rngx_initial_state: out is NULL");
    *out = rngx::init_state(rngx::seed_mix(seed), gid);
    return RNGX_OK;
}
