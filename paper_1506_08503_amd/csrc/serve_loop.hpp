// serve_loop.hpp -- the continuous-batching request loop of aes_serve_run,
// as host code with no HIP in it: admission, the batch cut, the output ring,
// the key-schedule cache and retirement.  The device side (staging, launches,
// completion queries, the clock) is a template parameter, so the same loop
// runs on the GPU (serve.hip) and against a simulated device in a CPU test.
//
// This is the per-row key and IV form of sec. II applied to requests that
// arrive over time: every request is one message with its own key, nonce and
// counter; batches of them are run by the batched persistent CTR kernel.
//
// One pass of the loop:
//   1. the requests whose arrival time has passed join the queue;
//   2. batches whose device work has completed retire, in submission order:
//      their requests are complete, the consumer is handed their results,
//      then their budget bytes, key-cache pins and output range are released;
//   3. queued requests that can never fit (input + output above the whole
//      budget, or an output larger than the whole output area) are rejected;
//   4. if a launch slot is free and either nothing runs, the queued payload
//      reaches max_batch_bytes, the oldest queued request has waited window_s
//      or the whole trace has arrived, the longest queue prefix that fits the
//      budget left, the free output range, max_batch_bytes (at least one
//      request), max_batch_reqs and the key cache becomes a batch;
//   5. if none of the above happened the device is told the loop is idle.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <limits>
#include <utility>
#include <vector>

#include "aesmi.h"
#include "serve_cache.hpp"

namespace aesmi {

inline uint64_t serve_pad16(uint64_t n) { return (n + 15u) & ~(uint64_t)15u; }

// Largest k <= kmax with cum[lo + k] - cum[lo] <= limit, for non-decreasing
// prefix sums cum.  The bound is compared as a difference (saturated), so a
// limit near 2^64 ("no limit") cannot wrap around.
inline uint64_t prefix_within(const std::vector<uint64_t> &cum, uint64_t lo, uint64_t kmax,
                              uint64_t limit)
{
    const uint64_t base = cum[lo];
    const uint64_t bound = limit > UINT64_MAX - base ? UINT64_MAX : base + limit;
    const auto first = cum.begin() + (ptrdiff_t)(lo + 1);
    return (uint64_t)(std::upper_bound(first, first + (ptrdiff_t)kmax, bound) - first);
}

// The output area as a ring.  Batches take contiguous ranges in submission
// order and give them back when they retire, in any order; space is reused
// once every range before it has been given back.  Ranges are never empty.
// Allocation moves forward and goes back to offset 0 only when the range
// does not fit before the end, so an area at least as large as all the
// outputs together is never reused.
struct OutRing {
    struct Range {
        uint64_t off, len;
        bool freed;
    };
    uint64_t cap;
    uint64_t head = 0;       // where the next range starts
    bool wrapped = false;    // live ranges run from the front range to cap, then from 0 to head
    uint64_t used = 0, peak = 0;
    std::deque<Range> live;  // in allocation order

    explicit OutRing(uint64_t capacity) : cap(capacity) {}

    // Longest range alloc() can hand out now.
    uint64_t max_alloc() const
    {
        if (live.empty())
            return cap;
        const uint64_t tail = live.front().off;
        if (wrapped)
            return tail - head;
        return std::max(cap - head, tail);
    }

    // Takes n (0 < n <= max_alloc()) bytes; returns the range's offset.
    uint64_t alloc(uint64_t n)
    {
        uint64_t off;
        if (live.empty()) {
            off = cap - head >= n ? head : 0;
            wrapped = false;
        } else if (!wrapped && cap - head >= n) {
            off = head;
        } else if (!wrapped) {
            off = 0;            // the bytes [head, cap) wait until the ring comes round
            wrapped = true;
        } else {
            off = head;
        }
        head = off + n;
        live.push_back(Range{off, n, false});
        used += n;
        peak = std::max(peak, used);
        return off;
    }

    // Gives back the range that starts at off.
    void release(uint64_t off)
    {
        for (Range &r : live)
            if (r.off == off && !r.freed) {
                r.freed = true;
                used -= r.len;
                break;
            }
        while (!live.empty() && live.front().freed)
            live.pop_front();
        if (live.empty()) {
            wrapped = false;    // all free; the next range still starts at head if it fits
        } else if (wrapped && live.front().off < head) {
            wrapped = false;    // every range left lies in [0, head)
        }
    }
};

// What the loop hands the device for one batch.  The segments (one per
// request, output offsets already set) were written into dev.segments(slot, k).
struct ServeBatchPlan {
    uint64_t first, count;   // requests [first, first + count)
    uint64_t out_base;       // offset of the batch's range in the output area
    uint64_t out_len;        // bytes of that range (the 16-padded outputs)
    const std::vector<std::pair<uint32_t, uint32_t>> *fills;   // (row, key) to expand
    uint32_t wait_mask;      // bit s: wait for slot s's key fills before reading rows
};

// The loop.  Dev provides
//   void start()                         start of the run: now() counts from here
//   double now()                         seconds since start()
//   int poll(uint32_t slot)              1 = the slot's batch has completed,
//                                        0 = not yet, < 0 = device error
//   aes_segment_t *segments(uint32_t slot, uint64_t k)   host room for the
//                                        k segments of the slot's next batch
//   int launch(uint32_t slot, const ServeBatchPlan &)   0 = enqueued, < 0 = error
//   void deliver(uint64_t first, uint64_t count)   results of a completed batch
//                                        are readable until this returns
//   void idle()                          called when a pass changed nothing
// The key cache kc may come from an earlier run on the same device (its
// rows are still expanded there; no row may be pinned); the hit and miss
// counts in stats are this run's.  Arguments were checked by the caller.
template <class Dev>
aes_status_t serve_loop(const aes_serve_request_t *reqs, size_t nreq,
                        const aes_serve_params_t &pr, uint64_t out_bytes, ServeKeyCache &kc,
                        Dev &dev, double *latency_s, uint64_t *out_off, aes_serve_stats_t *stats)
{
    const uint64_t hits0 = kc.hits, misses0 = kc.misses;
    const uint32_t nstreams = pr.nstreams, maxb = pr.max_batch_reqs;
    // Rows one batch may take from the unpinned ones: with the whole cache a
    // batch of a small cache pins every row and the next batch cannot start
    // until it ends; a share per stream lets batches overlap.
    const uint32_t row_cap = std::max<uint32_t>(1, pr.nslots / nstreams);
    // footprint = input + 16-padded output; prefix sums of footprint, output and payload
    std::vector<uint64_t> fp(nreq), cum_fp(nreq + 1, 0), cum_out(nreq + 1, 0),
        cum_b(nreq + 1, 0);
    std::vector<uint32_t> key_id(nreq);
    for (size_t i = 0; i < nreq; ++i) {
        fp[i] = reqs[i].nbytes + serve_pad16(reqs[i].nbytes);
        cum_fp[i + 1] = cum_fp[i] + fp[i];
        cum_out[i + 1] = cum_out[i] + serve_pad16(reqs[i].nbytes);
        cum_b[i + 1] = cum_b[i] + reqs[i].nbytes;
        key_id[i] = reqs[i].key_id;
        latency_s[i] = std::numeric_limits<double>::infinity();
        out_off[i] = UINT64_MAX;
    }

    struct InFlight {
        uint64_t first = 0, last = 0, held = 0, bytes = 0, out_base = 0;
        std::vector<uint32_t> rows, filled_rows;
    };
    std::vector<InFlight> slot(nstreams);
    std::vector<bool> busy(nstreams, false);
    std::deque<uint32_t> order;          // busy slots in submission order
    OutRing ring(out_bytes);
    // row -> slot whose in-flight batch expanded it (-1: none)
    std::vector<int32_t> filled_by(pr.nslots, -1);
    std::vector<uint32_t> keys;
    std::vector<std::pair<uint32_t, uint32_t>> fills;
    std::vector<double> complete(nreq, std::numeric_limits<double>::infinity());

    aes_serve_stats_t st{};
    uint64_t qh = 0, held = 0, arrived = pr.realtime ? 0 : nreq;
    const double window = pr.window_s;
    // the clock starts once the loop's own set-up is done: arrival times
    // count from here
    dev.start();
    while (qh < nreq || !order.empty()) {
        const double now = dev.now();
        bool progressed = false;
        while (arrived < nreq && reqs[arrived].arrival_s <= now)
            ++arrived;
        // retire finished batches, oldest first
        for (size_t j = 0; j < order.size();) {
            const uint32_t si = order[j];
            const int q = dev.poll(si);
            if (q < 0)
                return AES_ERR_HIP;
            if (q == 0) {
                ++j;
                continue;
            }
            InFlight &b = slot[si];
            const double tdone = dev.now();
            for (uint64_t i = b.first; i < b.last; ++i)
                complete[i] = tdone;
            dev.deliver(b.first, b.last - b.first);
            held -= b.held;
            kc.release(b.rows);
            ring.release(b.out_base);
            for (uint32_t row : b.filled_rows)
                if (filled_by[row] == (int32_t)si)
                    filled_by[row] = -1;
            st.completed += b.last - b.first;
            st.bytes += b.bytes;
            busy[si] = false;
            order.erase(order.begin() + (ptrdiff_t)j);
            progressed = true;
        }
        // reject what can never fit
        while (qh < arrived && (fp[qh] > pr.hbm_budget || serve_pad16(reqs[qh].nbytes) > out_bytes)) {
            ++st.rejected;
            ++qh;
            progressed = true;
        }
        if (qh < arrived && order.size() < nstreams) {
            const uint64_t queued = cum_b[arrived] - cum_b[qh];
            const double oldest = pr.realtime ? now - reqs[qh].arrival_s : 0.0;
            if (order.empty() || queued >= pr.max_batch_bytes || oldest >= window ||
                arrived == nreq) {
                const uint64_t avail = arrived - qh;
                uint64_t k = prefix_within(cum_fp, qh, avail, pr.hbm_budget - held);
                k = std::min(k, prefix_within(cum_out, qh, avail, ring.max_alloc()));
                const uint64_t kb = prefix_within(cum_b, qh, avail, pr.max_batch_bytes);
                k = std::min<uint64_t>({k, std::max<uint64_t>(kb, 1), (uint64_t)maxb});
                if (k)
                    k = kc.take(key_id.data() + qh, (uint32_t)k, row_cap, keys, fills);
                if (k) {
                    uint32_t si = 0;
                    while (busy[si])
                        ++si;
                    InFlight &b = slot[si];
                    // the rows this batch reads that another slot's in-flight
                    // batch is still expanding
                    uint32_t waits = 0;
                    for (uint32_t key : keys) {
                        const int32_t fb = filled_by[(uint32_t)kc.slot_of[key]];
                        if (fb >= 0 && fb != (int32_t)si)
                            waits |= 1u << fb;
                    }
                    const uint64_t out_len = cum_out[qh + k] - cum_out[qh];
                    const uint64_t base = ring.alloc(out_len);
                    aes_segment_t *sg = dev.segments(si, k);
                    uint64_t off = base;
                    for (uint64_t j = 0; j < k; ++j) {
                        const aes_serve_request_t &r = reqs[qh + j];
                        aes_segment_t &g = sg[j];
                        g.in_off = r.in_off;
                        g.out_off = off;
                        g.nbytes = r.nbytes;
                        g.key_slot = (uint32_t)kc.slot_of[r.key_id];
                        g.ctr0 = r.ctr0;
                        std::memcpy(g.nonce, r.nonce, 12);
                        g.reserved = 0;
                        out_off[qh + j] = off;
                        off += serve_pad16(r.nbytes);
                    }
                    b.filled_rows.clear();
                    for (const auto &f : fills) {
                        filled_by[f.first] = (int32_t)si;
                        b.filled_rows.push_back(f.first);
                    }
                    const ServeBatchPlan plan{qh, k, base, out_len, &fills, waits};
                    if (dev.launch(si, plan) < 0)
                        return AES_ERR_HIP;
                    b.rows.clear();
                    for (uint32_t key : keys)
                        b.rows.push_back((uint32_t)kc.slot_of[key]);
                    b.first = qh;
                    b.last = qh + k;
                    b.held = cum_fp[qh + k] - cum_fp[qh];
                    b.bytes = cum_b[qh + k] - cum_b[qh];
                    b.out_base = base;
                    busy[si] = true;
                    order.push_back(si);
                    held += b.held;
                    ++st.batches;
                    st.max_inflight = std::max<uint32_t>(st.max_inflight, (uint32_t)order.size());
                    st.max_held = std::max(st.max_held, held);
                    qh += k;
                    progressed = true;
                }
            }
        }
        if (!progressed)
            dev.idle();
    }
    st.elapsed_s = dev.now();
    for (size_t i = 0; i < nreq; ++i)
        if (std::isfinite(complete[i]))
            latency_s[i] = complete[i] - (pr.realtime ? reqs[i].arrival_s : 0.0);
    st.key_hits = kc.hits - hits0;
    st.key_misses = kc.misses - misses0;
    st.max_out_used = ring.peak;
    if (stats)
        *stats = st;
    return AES_OK;
}

}  // namespace aesmi
