// Model check of the request server's pool ring and ticket table (host-only
// header csrc/pool.h): random FIFO-ish admission/release sequences against a
// byte-map model of the pool. Exits non-zero on the first violation.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "pool.h"

struct Item {
    bool live = true;
    int v = 0;
};

static int fail(const char *what, long step)
{
    std::fprintf(stderr, "violation at step %ld: %s\n", step, what);
    return 1;
}

int main()
{
    // Exact scenario: two 400,000-byte blocks in a 1 MiB pool.
    {
        rngx::PoolRing r;
        r.reset(1 << 20);
        uint64_t o0, s0, o1, s1, o2, s2, o3, s3;
        if (!r.alloc(400000, &o0, &s0) || !r.alloc(400000, &o1, &s1))
            return fail("two blocks must fit", 0);
        if (r.alloc(400000, &o2, &s2))
            return fail("third block must not fit", 0);
        r.release(s0);
        if (!r.alloc(400000, &o2, &s2) || o2 != 0)
            return fail("third block must wrap to 0 after the first is freed", 0);
        if (r.alloc(400000, &o3, &s3))
            return fail("fourth block must wait for the second", 0);
        r.release(s1);
        if (!r.alloc(400000, &o3, &s3) || o3 != 400128)
            return fail("fourth block must follow the third", 0);
        r.release(s2);
        r.release(s3);
        if (r.used() != 0)
            return fail("pool must be empty", 0);
    }
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; ++trial) {
        const uint64_t cap = 256 * (64 + rng() % 4096);
        rngx::PoolRing r;
        r.reset(cap);
        std::vector<int> owner(cap / 256, -1); // granule -> block id
        struct Live {
            uint64_t off, size, seq;
            int id;
        };
        std::vector<Live> live;
        int next_id = 0;
        uint64_t model_used = 0;
        for (long step = 0; step < 4000; ++step) {
            const bool do_alloc = live.empty() || rng() % 100 < 55;
            if (do_alloc) {
                const uint64_t bytes = 1 + rng() % (cap / 3);
                uint64_t off, seq;
                if (!r.alloc(bytes, &off, &seq))
                    continue;
                const uint64_t size = (bytes + 255) & ~(uint64_t)255;
                if (off % 256 || off + size > cap)
                    return fail("block out of bounds or misaligned", step);
                for (uint64_t g = off / 256; g < (off + size) / 256; ++g) {
                    if (owner[g] != -1)
                        return fail("overlapping live blocks", step);
                    owner[g] = next_id;
                }
                live.push_back({off, size, seq, next_id++});
                model_used += size;
            } else {
                // Mostly the oldest block (FIFO), sometimes any block.
                size_t k = (rng() % 4 == 0) ? rng() % live.size() : 0;
                const Live b = live[k];
                live.erase(live.begin() + k);
                for (uint64_t g = b.off / 256; g < (b.off + b.size) / 256; ++g)
                    owner[g] = -1;
                model_used -= b.size;
                r.release(b.seq);
                r.release(b.seq); // double release is ignored
            }
            if (r.used() != model_used)
                return fail("used-byte count differs from the model", step);
            if (r.peak() < r.used())
                return fail("peak below used", step);
        }
        // Drain: everything freed returns the whole pool.
        for (const Live &b : live)
            r.release(b.seq);
        uint64_t off, seq;
        if (r.used() != 0 || !r.alloc(cap, &off, &seq) || off != 0)
            return fail("drained pool must hold one block of its full size", -1);
    }
    // Ticket table: consecutive tickets, erase in any order, front trimmed.
    {
        rngx::TicketTable<Item> t;
        t.clear(100);
        for (int i = 0; i < 50; ++i) {
            if (t.next_ticket() != 100u + i)
                return fail("tickets must be consecutive", i);
            t.add(Item{true, i});
        }
        for (int i = 49; i >= 0; i -= 2)
            t.erase(100 + i);
        for (int i = 0; i < 50; ++i) {
            Item *p = t.find(100 + i);
            if ((i % 2 == 1) != (p == nullptr) || (p && p->v != i))
                return fail("find after erase", i);
        }
        for (int i = 0; i < 50; i += 2)
            t.erase(100 + i);
        if (t.find(100) || t.find(149) || t.find(99) || t.next_ticket() != 150)
            return fail("table must be empty and keep numbering", 0);
    }
    std::printf("pool model check ok\n");
    return 0;
}
