// serve.hip -- the device side of aes_serve_run.
//
// The request loop itself (admission, batch cut, output ring, key cache,
// retirement) is host code in serve_loop.hpp; this file gives it a device:
// per-stream launch slots with pinned staging, the staging kernel that copies
// a batch's tables to the device and expands its missed keys, the batched
// T-table kernel, completion events and the clock.  A batch is one staging
// launch and one CTR launch on its slot's stream, so batches on different
// streams overlap on the device while the loop keeps admitting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "internal.hpp"
#include "serve_loop.hpp"

namespace aesmi {

// The loop's device.  Per stream slot: staging for one batch at a time, k
// requests with f key fills, in pinned host memory:
//   [workspace: header + tile_start[0..k]] [k segments] [f keys32 | f lens | f rows]
// the workspace written on the host (the prepare kernel is not launched).
// One kernel copies the workspace and the segments to the same offsets of
// the device staging and expands the fills straight from host memory.
class HipServeDevice {
public:
    HipServeDevice(const aes_serve_params_t &pr, const uint8_t *keys32, const uint8_t *key_len)
        : pr_(pr), keys32_(keys32), key_len_(key_len)
    {
        // waves of the batched kernel's grid (one 1,024-thread workgroup per CU)
        waves_ = 16u * (uint32_t)(device_cu_count() > 0 ? device_cu_count() : 256);
    }
    HipServeDevice(const HipServeDevice &) = delete;
    HipServeDevice &operator=(const HipServeDevice &) = delete;

    // The input pool and output area of the next run.
    void bind(const uint8_t *pool, uint8_t *out)
    {
        pool_ = pool;
        out_ = out;
    }

    ~HipServeDevice()
    {
        for (Slot &s : slots_)
            if (s.stream)
                (void)hipStreamSynchronize(s.stream);
        for (Slot &s : slots_) {
            if (s.done)
                (void)hipEventDestroy(s.done);
            if (s.filled)
                (void)hipEventDestroy(s.filled);
            if (s.stream)
                (void)hipStreamDestroy(s.stream);
            (void)hipHostFree(s.stage_h);
            (void)hipFree(s.stage_d);
        }
        (void)hipFree(table_);
    }

    // Key table, streams, events and staging for every run of this device.
    bool setup()
    {
        const uint32_t maxb = pr_.max_batch_reqs;
        const uint32_t nfill = std::min<uint32_t>(maxb, pr_.nslots);
        // the key cache's rows: nr, key_bytes and rk_enc are written on a
        // fill (counter mode reads nothing else)
        if (hipMalloc(&table_, sizeof(aes_key_schedule_t) * pr_.nslots) != hipSuccess)
            return false;
        const size_t stage_max = batched_workspace_bytes(maxb) +
                                 pad256(sizeof(aes_segment_t) * maxb) + fill_bytes(nfill);
        slots_.resize(pr_.nstreams);
        for (Slot &s : slots_) {
            if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&s.filled, hipEventDisableTiming) != hipSuccess ||
                hipHostMalloc((void **)&s.stage_h, stage_max, hipHostMallocMapped) != hipSuccess ||
                hipHostGetDevicePointer((void **)&s.stage_hd, s.stage_h, 0) != hipSuccess ||
                hipMalloc((void **)&s.stage_d, stage_max) != hipSuccess)
                return false;
        }
        return true;
    }

    void start() { t0_ = std::chrono::steady_clock::now(); }

    double now() const
    {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
    }

    int poll(uint32_t si)
    {
        const hipError_t q = hipEventQuery(slots_[si].done);
        if (q == hipErrorNotReady)
            return 0;
        return q == hipSuccess ? 1 : -1;
    }

    // The segments of a k-request batch go right after its workspace.
    aes_segment_t *segments(uint32_t si, uint64_t k)
    {
        return reinterpret_cast<aes_segment_t *>(slots_[si].stage_h +
                                                 batched_workspace_bytes((uint32_t)k));
    }

    int launch(uint32_t si, const ServeBatchPlan &p)
    {
        Slot &s = slots_[si];
        const uint32_t k = (uint32_t)p.count;
        const std::vector<std::pair<uint32_t, uint32_t>> &fills = *p.fills;
        for (uint32_t sj = 0; sj < pr_.nstreams; ++sj)
            if (((p.wait_mask >> sj) & 1u) &&
                hipStreamWaitEvent(s.stream, slots_[sj].filled, 0) != hipSuccess)
                return -1;
        // staging: workspace, segments (written by the loop), key fills
        const size_t ws_b = batched_workspace_bytes(k);
        const size_t seg_b = pad256(sizeof(aes_segment_t) * k);
        const aes_segment_t *sh = reinterpret_cast<const aes_segment_t *>(s.stage_h + ws_b);
        batched_prepare_host(sh, k, serve_tile(p.out_len >> 4, waves_), s.stage_h);
        const uint32_t f = (uint32_t)fills.size();
        uint8_t *kh = s.stage_h + ws_b + seg_b, *lh = kh + (size_t)f * 32;
        uint32_t *rh = reinterpret_cast<uint32_t *>(lh + ((f + 3u) & ~3u));
        for (uint32_t j = 0; j < f; ++j) {
            std::memcpy(kh + 32u * j, keys32_ + 32u * fills[j].second, 32);
            lh[j] = key_len_[fills[j].second];
            rh[j] = fills[j].first;
        }
        // workspace and segments to the device, key fills read from the
        // pinned staging: one launch
        const size_t fo = ws_b + seg_b;   // fills' offset in the staging
        const uint8_t *kd = s.stage_hd + fo, *ld = kd + (size_t)f * 32;
        const uint32_t *rd = reinterpret_cast<const uint32_t *>(ld + ((f + 3u) & ~3u));
        if (stage_and_expand(s.stage_hd, s.stage_d, fo, kd, ld, rd, f, table_, s.stream) !=
                hipSuccess ||
            (f && hipEventRecord(s.filled, s.stream) != hipSuccess))
            return -1;
        if (batched_ctr_prepared(reinterpret_cast<const aes_segment_t *>(s.stage_d + ws_b), k,
                                 table_, pool_, out_, s.stage_d, s.stream) != hipSuccess ||
            hipEventRecord(s.done, s.stream) != hipSuccess)
            return -1;
        return 0;
    }

    void deliver(uint64_t first, uint64_t count)
    {
        if (pr_.on_batch)
            pr_.on_batch(pr_.user, first, count);
    }

    void idle() {}

private:
    struct Slot {
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr, filled = nullptr;
        uint8_t *stage_h = nullptr;   // pinned, mapped
        uint8_t *stage_hd = nullptr;  // the same memory as the device addresses it
        uint8_t *stage_d = nullptr;
    };

    static size_t pad256(size_t n) { return (n + 255u) & ~(size_t)255u; }
    // Bytes of one fill staging area for up to f keys: keys32, lens, 4-aligned rows.
    static size_t fill_bytes(uint32_t f) { return (size_t)f * 32 + ((f + 3u) & ~3u) + (size_t)f * 4; }

    // Tile of the batched kernel for a serving batch of `blocks` blocks.  A
    // wave works through a tile alone, so a batch with fewer tiles than the
    // grid has waves takes as long as one wave's tile, and tiles claimed late
    // set the end of the launch: serving batches (up to 64 MiB by default,
    // i.e. up to about 1,024 blocks per wave) get 256-block tiles; batches
    // several times larger, where fewer tiles cost less per-tile set-up,
    // 1,024.  Measured, one 64 MiB batch of the lognormal request mix (2,160
    // requests, half AES-256): 256 / 512 / 1,024 / 2,048-block tiles 71.8 /
    // 79.1 / 80.7 / 115.5 us; in the 1,024-row closed loop 256, 512 and the
    // earlier rule (1,024 above 256 blocks per wave) all gave 33.7-34.1 M
    // requests/s, with p50/p99 at 80% load 0.088/0.157 ms for 256 against
    // 0.118/0.174 ms; 100 messages of 32 KiB take 20.1 us with 256-block
    // tiles and 33.8 us with 1,024.
    static uint32_t serve_tile(uint64_t blocks, uint32_t waves)
    {
        return blocks <= 2048ull * waves ? 256u : 1024u;
    }

    const aes_serve_params_t pr_;
    const uint8_t *keys32_, *key_len_;
    const uint8_t *pool_ = nullptr;
    uint8_t *out_ = nullptr;
    std::chrono::steady_clock::time_point t0_;
    uint32_t waves_ = 0;
    aes_key_schedule_t *table_ = nullptr;
    std::vector<Slot> slots_;
};

}  // namespace aesmi

// A server: the device of the loop (key table, streams, staging) and the key
// cache, set up once and used by every run.
struct aes_server {
    std::vector<uint8_t> keys32, key_len;
    aes_serve_params_t params;
    aesmi::ServeKeyCache cache;
    aesmi::HipServeDevice dev;

    aes_server(const aes_serve_params_t &pr, const uint8_t *k32, const uint8_t *klen, size_t nkeys)
        : keys32(k32, k32 + 32 * nkeys), key_len(klen, klen + nkeys), params(pr),
          cache(nkeys, pr.nslots), dev(pr, keys32.data(), key_len.data())
    {
    }
};

namespace aesmi {

aes_status_t server_create(const aes_serve_params_t &pr, const uint8_t *keys32,
                           const uint8_t *key_len, size_t nkeys, aes_server_t **out)
{
    aes_server_t *srv = new (std::nothrow) aes_server_t(pr, keys32, key_len, nkeys);
    if (!srv)
        return AES_ERR_HIP;
    if (!srv->dev.setup()) {
        delete srv;
        return AES_ERR_HIP;
    }
    *out = srv;
    return AES_OK;
}

aes_status_t server_run(aes_server_t *srv, const aes_serve_request_t *reqs, size_t nreq,
                        const uint8_t *pool, uint8_t *out, uint64_t out_bytes, double *latency_s,
                        uint64_t *out_off, aes_serve_stats_t *stats)
{
    srv->dev.bind(pool, out);
    return serve_loop(reqs, nreq, srv->params, out_bytes, srv->cache, srv->dev, latency_s,
                      out_off, stats);
}

void server_destroy(aes_server_t *srv)
{
    delete srv;
}

size_t server_nkeys(const aes_server_t *srv)
{
    return srv->key_len.size();
}

}  // namespace aesmi
