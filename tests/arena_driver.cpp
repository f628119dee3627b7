// Random allocation / release sequences on the serving arena's allocator,
// checked against a plain model (a byte map of the range): blocks never
// overlap, stay inside the range and aligned, the bytes in use match the
// model, an allocation fails only when no free run of that length exists,
// and releasing everything leaves one free range.  Prints "ok" or the first
// failure.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "tg_arena.hpp"

int main(int argc, char **argv) {
    const unsigned seed = argc > 1 ? (unsigned)atoi(argv[1]) : 1u;
    std::mt19937_64 rng(seed);
    const size_t size = 256 * 4096;
    tg::Arena a(size);
    std::vector<unsigned char> used(size / 256, 0);
    std::map<int64_t, size_t> live;
    for (int step = 0; step < 20000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t bytes = 1 + rng() % (256 * 300);
            const size_t units = (bytes + 255) / 256;
            const int64_t off = a.alloc(bytes);
            // model: is there a free run of `units`?
            size_t run = 0, best = 0;
            for (unsigned char u : used) {
                run = u ? 0 : run + 1;
                best = run > best ? run : best;
            }
            if (off < 0) {
                if (best >= units) { printf("alloc failed with a free run of %zu >= %zu\n", best, units); return 1; }
                continue;
            }
            if (off % 256 || (size_t)off + units * 256 > size) { printf("bad block %lld\n", (long long)off); return 1; }
            for (size_t q = 0; q < units; ++q) {
                if (used[off / 256 + q]) { printf("overlap at %lld\n", (long long)off); return 1; }
                used[off / 256 + q] = 1;
            }
            live[off] = units;
        } else {
            auto it = live.begin();
            std::advance(it, rng() % live.size());
            if (!a.release(it->first)) { printf("release refused\n"); return 1; }
            for (size_t q = 0; q < it->second; ++q) used[it->first / 256 + q] = 0;
            live.erase(it);
        }
        size_t model = 0;
        for (unsigned char u : used) model += u;
        if (a.in_use() != model * 256) { printf("in_use %zu != %zu\n", a.in_use(), model * 256); return 1; }
    }
    if (a.release(12345)) { printf("released a non-block\n"); return 1; }
    for (auto &b : live) a.release(b.first);
    if (a.in_use() != 0 || a.free_ranges() != 1 || a.largest_free() != size) {
        printf("not whole after releasing everything\n");
        return 1;
    }
    printf("ok\n");
    return 0;
}
