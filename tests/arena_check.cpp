// Random allocate / release sequences on the serving loop's arena allocator,
// checked against a plain bitmap of the arena: every placement is the lowest
// offset with a free run of the requested length (first fit), a request
// fails exactly when no such run exists, placements never overlap, and the
// free list holds exactly the unused granules, as maximal runs.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "hr_arena.h"

static int fail(const char* what, long a, long b)
{
    std::printf("FAIL %s %ld %ld\n", what, a, b);
    return 1;
}

int main(int argc, char** argv)
{
    const uint64_t size = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 512;
    const int steps = argc > 2 ? std::atoi(argv[2]) : 20000;
    std::mt19937_64 rng(argc > 3 ? std::strtoull(argv[3], nullptr, 10) : 1);
    arena_alloc a(size);
    std::vector<char> used(size, 0);
    struct blk { uint64_t off, n; };
    std::vector<blk> live;
    for (int s = 0; s < steps; ++s) {
        if (live.empty() || rng() % 100 < 55) {
            const uint64_t n = 1 + rng() % (rng() % 4 == 0 ? size / 2 : 16);
            // expected first fit from the bitmap
            long want = -1;
            for (uint64_t o = 0, run = 0; o < size; ++o) {
                run = used[o] ? 0 : run + 1;
                if (run == n) { want = (long)(o + 1 - n); break; }
            }
            uint64_t off = 0;
            const bool ok = a.alloc(n, &off);
            if (ok != (want >= 0)) return fail("alloc result", ok, want);
            if (ok) {
                if ((long)off != want) return fail("first fit", (long)off, want);
                for (uint64_t i = off; i < off + n; ++i) used[i] = 1;
                live.push_back({off, n});
            }
        } else {
            const size_t k = rng() % live.size();
            a.release(live[k].off, live[k].n);
            for (uint64_t i = live[k].off; i < live[k].off + live[k].n; ++i) used[i] = 0;
            live[k] = live.back();
            live.pop_back();
        }
        // the free list is exactly the unused granules, as maximal runs
        uint64_t pos = 0, prev_end = UINT64_MAX;
        for (const auto& f : a.free_) {
            if (f.second == 0) return fail("empty run", (long)f.first, 0);
            if (f.first == prev_end) return fail("adjacent runs", (long)f.first, 0);
            for (; pos < f.first; ++pos)
                if (!used[pos]) return fail("free granule not listed", (long)pos, s);
            for (; pos < f.first + f.second; ++pos)
                if (used[pos]) return fail("listed granule in use", (long)pos, s);
            prev_end = f.first + f.second;
        }
        for (; pos < size; ++pos)
            if (!used[pos]) return fail("free granule not listed", (long)pos, s);
    }
    std::printf("ok %zu live\n", live.size());
    return 0;
}
