// serve_cache.hpp -- the key-schedule cache of the serving loop (host code,
// no HIP): which key's schedule sits in which row of the device table.
//
// A batch is a prefix of the queued requests.  take() finds the longest
// prefix whose distinct keys fit, pins their rows and names the rows that
// must be (re)expanded; release() unpins a finished batch's rows.  Victims
// for missing keys are unpinned rows that the batch does not hit: empty rows
// first, then the least recently used (ties by row index), assigned to the
// missing keys in ascending key order.
#pragma once

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

namespace aesmi {

// Which key sits in which row of the device schedule table.  A row is pinned
// once per in-flight batch that uses it and is never evicted while pinned.
struct ServeKeyCache {
    std::vector<int64_t> slot_of;    // per key: row or -1
    std::vector<int64_t> key_of;     // per row: key or -1
    std::vector<uint64_t> last_use;  // per row
    std::vector<uint32_t> pins;      // per row
    std::vector<uint64_t> seen;      // per key: stamp of the batch being formed
    std::vector<uint64_t> missed;    // per key: stamp when it missed in that batch
    std::vector<uint64_t> hit_row;   // per row: stamp when a key of that batch hit it
    uint64_t tick = 0, stamp = 0, hits = 0, misses = 0;
    uint32_t unpinned = 0;
    std::vector<uint64_t> cand;      // scratch of take(): victim candidates
    std::vector<uint32_t> missing;   // scratch of take(): keys to fill

    ServeKeyCache(size_t nkeys, uint32_t nslots)
        : slot_of(nkeys, -1), key_of(nslots, -1), last_use(nslots, 0), pins(nslots, 0),
          seen(nkeys, 0), missed(nkeys, 0), hit_row(nslots, 0), unpinned(nslots)
    {
    }

    // Largest k <= kmax such that the distinct keys of requests [0, k) fit:
    // every key that misses, and every key that hits an unpinned row, needs
    // one of the unpinned rows, and at most row_cap of them are taken.  Then
    // pins (and fills) the rows of that prefix.  Returns k (0: not even the
    // first request fits now); `keys` gets the prefix's distinct keys,
    // `fills` the (row, key) pairs to expand.
    uint32_t take(const uint32_t *key_id, uint32_t kmax, uint32_t row_cap,
                  std::vector<uint32_t> &keys, std::vector<std::pair<uint32_t, uint32_t>> &fills)
    {
        ++stamp;
        keys.clear();
        fills.clear();
        uint32_t need = 0, k = 0;
        for (; k < kmax; ++k) {
            const uint32_t key = key_id[k];
            if (seen[key] == stamp)
                continue;
            const int64_t row = slot_of[key];
            const bool takes = row < 0 || pins[row] == 0;
            if (takes && (need + 1 > unpinned || need + 1 > row_cap))
                break;
            seen[key] = stamp;
            need += takes;
            keys.push_back(key);
        }
        if (k == 0)
            return 0;
        // rows this batch hits are not eviction candidates
        uint32_t nmiss = 0;
        for (uint32_t key : keys) {
            if (slot_of[key] >= 0)
                hit_row[slot_of[key]] = stamp;
            else
                ++nmiss;
        }
        if (nmiss) {
            // victims: empty rows first, then the least recently used, ties
            // by row.  A row is empty exactly while its last_use is 0 (rows
            // are refilled, never emptied, and ticks start at 1), so that
            // order is the order of last_use << 32 | row.
            cand.clear();
            for (uint32_t r = 0; r < key_of.size(); ++r)
                if (pins[r] == 0 && hit_row[r] != stamp)
                    cand.push_back(last_use[r] << 32 | r);
            std::partial_sort(cand.begin(), cand.begin() + nmiss, cand.end());
            // the missing keys take them in ascending key order
            missing.clear();
            for (uint32_t key : keys)
                if (slot_of[key] < 0)
                    missing.push_back(key);
            std::sort(missing.begin(), missing.end());
            uint32_t v = 0;
            for (uint32_t key : missing) {
                const uint32_t row = (uint32_t)cand[v++];
                if (key_of[row] >= 0)
                    slot_of[key_of[row]] = -1;
                key_of[row] = key;
                slot_of[key] = row;
                missed[key] = stamp;
                fills.emplace_back(row, key);
            }
        }
        ++tick;
        for (uint32_t key : keys) {
            const uint32_t row = (uint32_t)slot_of[key];
            last_use[row] = tick;
            if (pins[row]++ == 0)
                --unpinned;
        }
        for (uint32_t i = 0; i < k; ++i) {
            if (missed[key_id[i]] == stamp)
                ++misses;
            else
                ++hits;
        }
        return k;
    }

    void release(const std::vector<uint32_t> &rows)
    {
        for (uint32_t row : rows)
            if (--pins[row] == 0)
                ++unpinned;
    }
};

}  // namespace aesmi
