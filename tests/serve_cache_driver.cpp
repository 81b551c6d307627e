// Runs the serving loop's key cache (csrc/serve_cache.hpp) on commands read
// from stdin, for the host tests:
//   first line: nkeys nslots
//   T cap n id_0 .. id_(n-1)   take a batch from these queued requests
//   R b                        release the rows of the b-th take
//   S                          print the row of every key
// Each T prints "T k hits misses nfills row key row key ..." (totals so far).
#include <cstdio>
#include <utility>
#include <vector>

#include "serve_cache.hpp"

int main()
{
    size_t nkeys = 0;
    unsigned nslots = 0;
    if (std::scanf("%zu %u", &nkeys, &nslots) != 2)
        return 1;
    aesmi::ServeKeyCache kc(nkeys, nslots);
    std::vector<std::vector<uint32_t>> taken;
    char op = 0;
    while (std::scanf(" %c", &op) == 1) {
        if (op == 'T') {
            unsigned cap = 0, n = 0;
            if (std::scanf("%u %u", &cap, &n) != 2)
                return 1;
            std::vector<uint32_t> ids(n);
            for (uint32_t &x : ids)
                if (std::scanf("%u", &x) != 1 || x >= nkeys)
                    return 1;
            std::vector<uint32_t> keys;
            std::vector<std::pair<uint32_t, uint32_t>> fills;
            const uint32_t k = kc.take(ids.data(), n, cap, keys, fills);
            std::vector<uint32_t> rows;
            for (uint32_t key : keys)
                rows.push_back((uint32_t)kc.slot_of[key]);
            taken.push_back(rows);
            std::printf("T %u %llu %llu %zu", k, (unsigned long long)kc.hits,
                        (unsigned long long)kc.misses, fills.size());
            for (const auto &f : fills)
                std::printf(" %u %u", f.first, f.second);
            std::printf("\n");
        } else if (op == 'R') {
            unsigned b = 0;
            if (std::scanf("%u", &b) != 1 || b >= taken.size())
                return 1;
            kc.release(taken[b]);
        } else if (op == 'S') {
            for (size_t key = 0; key < nkeys; ++key)
                std::printf("%lld ", (long long)kc.slot_of[key]);
            std::printf("\n");
        } else {
            return 1;
        }
    }
    return 0;
}
