// Runs the serving loop (csrc/serve_loop.hpp) on the CPU against a simulated
// device, for the host tests.  Two modes, chosen by the first word on stdin:
//
//   loop nreq nkeys nslots nstreams max_batch_reqs realtime hbm_budget
//        max_batch_bytes window_s out_bytes latency_s rate_Bps tick_s
//   then nreq lines "arrival_s nbytes key_id"
//     The simulated device runs one batch at a time in submission order: a
//     batch submitted at time t completes at max(t, previous completion) +
//     latency_s + payload bytes / rate_Bps; time moves only when the loop
//     reports a pass with no progress (by tick_s).  Prints one line per batch
//     "B first count out_base nfills row key row key ...", then
//     "L latency" per request (%.17g), then
//     "S completed rejected batches bytes hits misses max_held max_out_used max_inflight".
//
//   ring cap nops, then nops lines "A n" (allocate n bytes, prints the offset,
//     or -1 when n > max_alloc()) or "F i" (give back the range of the i-th
//     allocation; nothing for one that failed); prints max_alloc() after
//     every operation as "M value".
#include <cstdio>
#include <cstring>
#include <utility>
#include <vector>

#include "serve_loop.hpp"

namespace {

struct SimDevice {
    double t = 0, next_free = 0, latency = 0, rate = 1, tick = 1e-6;
    const aes_serve_request_t *reqs = nullptr;
    std::vector<double> done_at;
    std::vector<std::vector<aes_segment_t>> segs;

    void start() {}
    double now() const { return t; }
    int poll(uint32_t si) const { return t >= done_at[si] ? 1 : 0; }
    aes_segment_t *segments(uint32_t si, uint64_t k)
    {
        segs[si].resize(k);
        return segs[si].data();
    }
    int launch(uint32_t si, const aesmi::ServeBatchPlan &p)
    {
        uint64_t bytes = 0;
        for (uint64_t i = p.first; i < p.first + p.count; ++i)
            bytes += reqs[i].nbytes;
        const double start = t > next_free ? t : next_free;
        done_at[si] = start + latency + (double)bytes / rate;
        next_free = done_at[si];
        std::printf("B %llu %llu %llu %zu", (unsigned long long)p.first,
                    (unsigned long long)p.count, (unsigned long long)p.out_base, p.fills->size());
        for (const auto &f : *p.fills)
            std::printf(" %u %u", f.first, f.second);
        std::printf("\n");
        return 0;
    }
    void deliver(uint64_t, uint64_t) {}
    void idle() { t += tick; }
};

int run_loop()
{
    unsigned long long nreq, nkeys, budget, max_bytes, out_bytes;
    unsigned nslots, nstreams, maxb, realtime;
    double window, latency, rate, tick;
    if (std::scanf("%llu %llu %u %u %u %u %llu %llu %lf %llu %lf %lf %lf", &nreq, &nkeys,
                   &nslots, &nstreams, &maxb, &realtime, &budget, &max_bytes, &window,
                   &out_bytes, &latency, &rate, &tick) != 13)
        return 1;
    std::vector<aes_serve_request_t> reqs(nreq);
    for (auto &r : reqs) {
        std::memset(&r, 0, sizeof r);
        unsigned long long nb;
        unsigned kid;
        if (std::scanf("%lf %llu %u", &r.arrival_s, &nb, &kid) != 3 || kid >= nkeys)
            return 1;
        r.nbytes = nb;
        r.key_id = kid;
    }
    aes_serve_params_t pr{};
    pr.nslots = nslots;
    pr.nstreams = nstreams;
    pr.max_batch_reqs = maxb;
    pr.realtime = realtime;
    pr.hbm_budget = budget;
    pr.max_batch_bytes = max_bytes;
    pr.window_s = window;
    SimDevice dev;
    dev.latency = latency;
    dev.rate = rate;
    dev.tick = tick;
    dev.reqs = reqs.data();
    dev.done_at.assign(nstreams, 0.0);
    dev.segs.resize(nstreams);
    std::vector<double> lat(nreq);
    std::vector<uint64_t> off(nreq);
    aes_serve_stats_t st{};
    aesmi::ServeKeyCache kc(nkeys, nslots);
    if (aesmi::serve_loop(reqs.data(), nreq, pr, out_bytes, kc, dev, lat.data(), off.data(),
                          &st) != AES_OK)
        return 2;
    for (double v : lat)
        std::printf("L %.17g\n", v);
    std::printf("S %llu %llu %llu %llu %llu %llu %llu %llu %u\n",
                (unsigned long long)st.completed, (unsigned long long)st.rejected,
                (unsigned long long)st.batches, (unsigned long long)st.bytes,
                (unsigned long long)st.key_hits, (unsigned long long)st.key_misses,
                (unsigned long long)st.max_held, (unsigned long long)st.max_out_used,
                st.max_inflight);
    return 0;
}

int run_ring()
{
    unsigned long long cap, nops;
    if (std::scanf("%llu %llu", &cap, &nops) != 2)
        return 1;
    aesmi::OutRing ring(cap);
    std::vector<unsigned long long> offs;
    for (unsigned long long i = 0; i < nops; ++i) {
        char op = 0;
        unsigned long long v = 0;
        if (std::scanf(" %c %llu", &op, &v) != 2)
            return 1;
        if (op == 'A') {
            if (v == 0 || v > ring.max_alloc()) {
                std::printf("A -1\n");
                offs.push_back(~0ull);
            } else {
                offs.push_back(ring.alloc(v));
                std::printf("A %llu\n", offs.back());
            }
        } else if (op == 'F') {
            if (v >= offs.size())
                return 1;
            if (offs[v] != ~0ull)   // a failed allocation has nothing to give back
                ring.release(offs[v]);
        } else {
            return 1;
        }
        std::printf("M %llu\n", (unsigned long long)ring.max_alloc());
    }
    return 0;
}

}  // namespace

int main()
{
    char mode[16] = {0};
    if (std::scanf("%15s", mode) != 1)
        return 1;
    if (!std::strcmp(mode, "loop"))
        return run_loop();
    if (!std::strcmp(mode, "ring"))
        return run_ring();
    return 1;
}
