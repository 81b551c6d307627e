// serve.hip -- the continuous-batching request loop behind aes_serve_run.
//
// Host code only: it plays a trace of CTR requests (arrival time, payload in
// a device pool, key id, nonce, first counter) against the device.  Requests
// are admitted in arrival order under an HBM budget, their key schedules are
// kept in a device cache (LRU among rows that no in-flight batch uses,
// misses expanded on the device into their rows), and queued requests are
// closed into batches, each run by the batched persistent CTR kernel on one
// of a few streams, so that batches overlap on the device while the loop
// keeps admitting.  The loop writes each batch's tile table itself (it holds
// the segments anyway), so a batch is one host-to-device copy, the key
// expansion when keys missed, and one kernel.  This is the per-row key and IV form of sec. II applied to
// requests that arrive over time.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "internal.hpp"
#include "serve_cache.hpp"

namespace aesmi {
namespace {

// Per-stream launch slot: staging for one batch at a time, k requests with f
// key fills, in pinned host memory:
//   [workspace: header + tile_start[0..k]] [k segments] [f keys32 | f lens | f rows]
// the workspace written on the host (the prepare kernel is not launched).
// One kernel copies the workspace and the segments to the same offsets of
// the device staging and expands the fills straight from host memory.
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr, filled = nullptr;
    uint8_t *stage_h = nullptr;   // pinned, mapped
    uint8_t *stage_hd = nullptr;  // the same memory as the device addresses it
    uint8_t *stage_d = nullptr;
    bool busy = false;
    // the batch in flight
    uint64_t first = 0, last = 0, held = 0, bytes = 0;
    std::vector<uint32_t> rows, filled_rows;
};

struct Resources {
    aes_key_schedule_t *table = nullptr;
    std::vector<Slot> slots;
    ~Resources()
    {
        for (Slot &s : slots) {
            if (s.stream)
                (void)hipStreamSynchronize(s.stream);
        }
        for (Slot &s : slots) {
            if (s.done)
                (void)hipEventDestroy(s.done);
            if (s.filled)
                (void)hipEventDestroy(s.filled);
            if (s.stream)
                (void)hipStreamDestroy(s.stream);
            (void)hipHostFree(s.stage_h);
            (void)hipFree(s.stage_d);
        }
        (void)hipFree(table);
    }
};

// Tile of the batched kernel for a serving batch of `blocks` blocks.  A wave
// works through a tile alone, so a batch with fewer tiles than the grid has
// waves takes as long as one wave's tile: small batches get small tiles.
// Large ones keep 1,024 blocks, where fewer tiles cost less per-tile set-up.
// Measured (1,024 key rows, lognormal mix, median 4 KiB): 1,024-block tiles
// 26.3-27.0 M requests/s closed loop and p50/p99 0.088/0.116 ms at 8 M
// requests/s offered (batches of ~400, ~12 MB); 256-block tiles 22.4 M/s but
// p50 0.065 ms at 8 M/s, and p99 0.22 ms at 14 M/s; 100 messages of 32 KiB
// take 33.8 us with 1,024-block tiles and 20.1 us with 256.
inline uint32_t serve_tile(uint64_t blocks, uint32_t waves)
{
    if (blocks <= 128ull * waves)
        return 256;
    if (blocks <= 256ull * waves)
        return 512;
    return 1024;
}

inline uint64_t pad16(uint64_t n) { return (n + 15u) & ~(uint64_t)15u; }
inline size_t pad256(size_t n) { return (n + 255u) & ~(size_t)255u; }

// Bytes of one fill staging area for up to f keys: keys32, lens, 4-aligned rows.
inline size_t fill_bytes(uint32_t f) { return (size_t)f * 32 + ((f + 3u) & ~3u) + (size_t)f * 4; }

}  // namespace

aes_status_t serve_run(const aes_serve_request_t *reqs, size_t nreq, const uint8_t *keys32,
                       const uint8_t *key_len, size_t nkeys, const uint8_t *pool, uint8_t *out,
                       const aes_serve_params_t &pr, double *latency_s, uint64_t *out_off,
                       aes_serve_stats_t *stats)
{
    using clock = std::chrono::steady_clock;
    const uint32_t nstreams = pr.nstreams, maxb = pr.max_batch_reqs;
    const uint32_t nfill = std::min<uint32_t>(maxb, pr.nslots);
    // Rows one batch may take from the unpinned ones: with the whole cache a
    // batch of a small cache pins every row and the next batch cannot start
    // until it ends; a share per stream lets batches overlap.
    const uint32_t row_cap = std::max<uint32_t>(1, pr.nslots / nstreams);
    // waves of the batched kernel's grid (one 1,024-thread workgroup per CU)
    const uint32_t waves = 16u * (uint32_t)(device_cu_count() > 0 ? device_cu_count() : 256);
    // footprint = input + 16-padded output; prefix sums of footprint and bytes
    std::vector<uint64_t> fp(nreq), cum_fp(nreq + 1, 0), cum_b(nreq + 1, 0);
    std::vector<uint32_t> key_id(nreq);
    for (size_t i = 0; i < nreq; ++i) {
        fp[i] = reqs[i].nbytes + pad16(reqs[i].nbytes);
        cum_fp[i + 1] = cum_fp[i] + fp[i];
        cum_b[i + 1] = cum_b[i] + reqs[i].nbytes;
        key_id[i] = reqs[i].key_id;
        latency_s[i] = std::numeric_limits<double>::infinity();
        out_off[i] = UINT64_MAX;
    }

    Resources res;
    ServeKeyCache kc(nkeys, pr.nslots);
    // the key cache's rows: nr, key_bytes and rk_enc are written on a fill
    // (counter mode reads nothing else)
    if (hipMalloc(&res.table, sizeof(aes_key_schedule_t) * pr.nslots) != hipSuccess)
        return AES_ERR_HIP;
    const size_t stage_max = batched_workspace_bytes(maxb) +
                             pad256(sizeof(aes_segment_t) * maxb) + fill_bytes(nfill);
    res.slots.resize(nstreams);
    for (Slot &s : res.slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&s.filled, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&s.stage_h, stage_max, hipHostMallocMapped) != hipSuccess ||
            hipHostGetDevicePointer((void **)&s.stage_hd, s.stage_h, 0) != hipSuccess ||
            hipMalloc((void **)&s.stage_d, stage_max) != hipSuccess)
            return AES_ERR_HIP;
        s.rows.reserve(pr.nslots);
    }
    // row -> stream slot whose in-flight batch expanded it (-1: none)
    std::vector<int32_t> filled_by(pr.nslots, -1);
    std::vector<uint32_t> keys;
    std::vector<std::pair<uint32_t, uint32_t>> fills;
    std::vector<double> complete(nreq, std::numeric_limits<double>::infinity());

    aes_serve_stats_t st{};
    uint64_t qh = 0, held = 0, arena = 0;
    uint32_t inflight = 0;
    const double window = pr.window_s;
    const auto t0 = clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(clock::now() - t0).count(); };

    uint64_t arrived = pr.realtime ? 0 : nreq;
    while (qh < nreq || inflight) {
        const double now = now_s();
        // requests are sorted by arrival time
        while (arrived < nreq && reqs[arrived].arrival_s <= now)
            ++arrived;
        // retire finished batches
        for (uint32_t si = 0; si < nstreams; ++si) {
            Slot &s = res.slots[si];
            if (!s.busy)
                continue;
            const hipError_t q = hipEventQuery(s.done);
            if (q == hipErrorNotReady)
                continue;
            if (q != hipSuccess)
                return AES_ERR_HIP;
            const double tdone = now_s();
            for (uint64_t i = s.first; i < s.last; ++i)
                complete[i] = tdone;
            held -= s.held;
            kc.release(s.rows);
            for (uint32_t row : s.filled_rows)
                if (filled_by[row] == (int32_t)si)
                    filled_by[row] = -1;
            st.completed += s.last - s.first;
            st.bytes += s.bytes;
            s.busy = false;
            --inflight;
        }
        // reject what can never fit
        while (qh < arrived && fp[qh] > pr.hbm_budget) {
            ++st.rejected;
            ++qh;
        }
        if (qh < arrived && inflight < nstreams) {
            const uint64_t queued = cum_b[arrived] - cum_b[qh];
            const double oldest = pr.realtime ? now - reqs[qh].arrival_s : 0.0;
            if (!inflight || queued >= pr.max_batch_bytes || oldest >= window || arrived == nreq) {
                // largest prefix within the budget, the batch size limits and
                // the key cache
                const uint64_t room = pr.hbm_budget - held;
                uint64_t k = std::upper_bound(cum_fp.begin() + qh + 1, cum_fp.begin() + arrived + 1,
                                              cum_fp[qh] + room) - (cum_fp.begin() + qh + 1);
                uint64_t kb = std::upper_bound(cum_b.begin() + qh + 1, cum_b.begin() + arrived + 1,
                                               cum_b[qh] + pr.max_batch_bytes) -
                              (cum_b.begin() + qh + 1);
                k = std::min<uint64_t>({k, std::max<uint64_t>(kb, 1), maxb, arrived - qh});
                if (k)
                    k = kc.take(key_id.data() + qh, (uint32_t)k, row_cap, keys, fills);
                if (k) {
                    uint32_t si = 0;
                    while (res.slots[si].busy)
                        ++si;
                    Slot &s = res.slots[si];
                    // the rows this batch reads that another stream's
                    // in-flight batch is still expanding
                    bool waits[kServeMaxStreams] = {};
                    for (uint32_t key : keys) {
                        const int32_t fb = filled_by[(uint32_t)kc.slot_of[key]];
                        if (fb >= 0 && fb != (int32_t)si)
                            waits[fb] = true;
                    }
                    for (uint32_t sj = 0; sj < nstreams; ++sj)
                        if (waits[sj] &&
                            hipStreamWaitEvent(s.stream, res.slots[sj].filled, 0) != hipSuccess)
                            return AES_ERR_HIP;
                    // staging: workspace, segments, key fills
                    const size_t ws_b = batched_workspace_bytes((uint32_t)k);
                    const size_t seg_b = pad256(sizeof(aes_segment_t) * k);
                    const uint32_t f = (uint32_t)fills.size();
                    aes_segment_t *sh = reinterpret_cast<aes_segment_t *>(s.stage_h + ws_b);
                    uint64_t off = 0;
                    for (uint64_t j = 0; j < k; ++j) {
                        const aes_serve_request_t &r = reqs[qh + j];
                        aes_segment_t &g = sh[j];
                        g.in_off = r.in_off;
                        g.out_off = arena + off;
                        g.nbytes = r.nbytes;
                        g.key_slot = (uint32_t)kc.slot_of[r.key_id];
                        g.ctr0 = r.ctr0;
                        std::memcpy(g.nonce, r.nonce, 12);
                        g.reserved = 0;
                        out_off[qh + j] = arena + off;
                        off += pad16(r.nbytes);
                    }
                    batched_prepare_host(sh, (uint32_t)k, serve_tile(off >> 4, waves), s.stage_h);
                    s.filled_rows.clear();
                    uint8_t *kh = s.stage_h + ws_b + seg_b, *lh = kh + (size_t)f * 32;
                    uint32_t *rh = reinterpret_cast<uint32_t *>(lh + ((f + 3u) & ~3u));
                    for (uint32_t j = 0; j < f; ++j) {
                        std::memcpy(kh + 32u * j, keys32 + 32u * fills[j].second, 32);
                        lh[j] = key_len[fills[j].second];
                        rh[j] = fills[j].first;
                        filled_by[fills[j].first] = (int32_t)si;
                        s.filled_rows.push_back(fills[j].first);
                    }
                    // workspace and segments to the device, key fills read
                    // from the pinned staging: one launch
                    const size_t fo = ws_b + seg_b;   // fills' offset in the staging
                    const uint8_t *kd = s.stage_hd + fo, *ld = kd + (size_t)f * 32;
                    const uint32_t *rd = reinterpret_cast<const uint32_t *>(ld + ((f + 3u) & ~3u));
                    if (stage_and_expand(s.stage_hd, s.stage_d, fo, kd, ld, rd, f, res.table,
                                         s.stream) != hipSuccess ||
                        (f && hipEventRecord(s.filled, s.stream) != hipSuccess))
                        return AES_ERR_HIP;
                    if (batched_ctr_prepared(reinterpret_cast<const aes_segment_t *>(s.stage_d + ws_b),
                                             (uint32_t)k, res.table, pool, out, s.stage_d,
                                             s.stream) != hipSuccess ||
                        hipEventRecord(s.done, s.stream) != hipSuccess)
                        return AES_ERR_HIP;
                    arena += off;
                    s.rows.clear();
                    for (uint32_t key : keys)
                        s.rows.push_back((uint32_t)kc.slot_of[key]);
                    s.first = qh;
                    s.last = qh + k;
                    s.held = cum_fp[qh + k] - cum_fp[qh];
                    s.bytes = cum_b[qh + k] - cum_b[qh];
                    s.busy = true;
                    held += s.held;
                    ++inflight;
                    ++st.batches;
                    st.max_inflight = std::max(st.max_inflight, inflight);
                    st.max_held = std::max(st.max_held, held);
                    qh += k;
                }
            }
        }
    }
    st.elapsed_s = now_s();
    for (size_t i = 0; i < nreq; ++i)
        if (std::isfinite(complete[i]))
            latency_s[i] = complete[i] - (pr.realtime ? reqs[i].arrival_s : 0.0);
    st.key_hits = kc.hits;
    st.key_misses = kc.misses;
    if (stats)
        *stats = st;
    return AES_OK;
}

}  // namespace aesmi
