// Randomised check of the serving arena against a brute-force occupancy map.
#include <cassert>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_1207_5558_amd/csrc/arena.h"

int main() {
    const size_t align = 256, cap = 256 * 1000;
    slsht::Arena a(cap, align);
    std::vector<char> used(cap / align, 0);
    std::vector<std::pair<size_t, size_t>> live;   // (offset, rounded size)
    std::mt19937_64 rng(12345);
    size_t allocs = 0, fails = 0;
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t n = 1 + rng() % (align * 40);
            const size_t off = a.alloc(n);
            const size_t need = (n + align - 1) / align * align;
            if (off == slsht::Arena::kFail) {
                // first fit failed: no free run of need/align slots may exist
                size_t run = 0, best = 0;
                for (char u : used) { run = u ? 0 : run + 1; best = run > best ? run : best; }
                assert(best * align < need);
                assert(a.largest_free() < need);
                ++fails;
                continue;
            }
            assert(off % align == 0 && off + need <= cap);
            for (size_t k = off / align; k < (off + need) / align; ++k) { assert(!used[k]); used[k] = 1; }
            live.push_back({off, need});
            ++allocs;
        } else {
            const size_t i = rng() % live.size();
            assert(a.release(live[i].first));
            for (size_t k = live[i].first / align; k < (live[i].first + live[i].second) / align; ++k) used[k] = 0;
            live[i] = live.back();
            live.pop_back();
        }
        size_t u = 0;
        for (auto& p : live) u += p.second;
        assert(a.used() == u);
        assert(a.live_blocks() == live.size());
    }
    assert(!a.release(1));                 // not a block start
    for (auto& p : live) assert(a.release(p.first));
    assert(a.used() == 0 && a.free_ranges() == 1 && a.largest_free() == cap);
    assert(a.alloc(cap) == 0 && a.alloc(1) == slsht::Arena::kFail);
    printf("arena ok: %zu allocations, %zu first-fit misses\n", allocs, fails);
    return 0;
}
