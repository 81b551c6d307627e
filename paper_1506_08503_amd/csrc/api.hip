// api.hip -- the C ABI of libaesmi: argument validation, dispatch to the
// kernels, host key expansion and the batched-graph object.
#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>
#include <new>
#include <string.h>

#include "aes_tables.hpp"
#include "aesmi.h"
#include "internal.hpp"
#include "keysched.hpp"

namespace aesmi {

int device_cu_count()
{
    static std::mutex mu;
    static int cached[64];
    static bool init = false;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return 0;
    std::lock_guard<std::mutex> lock(mu);
    if (!init) {
        for (int &c : cached)
            c = -1;
        init = true;
    }
    if (cached[dev] < 0) {
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            cu = 0;
        cached[dev] = cu;
    }
    return cached[dev];
}

aes_status_t expand_key_host(const uint8_t *key, size_t key_bytes, aes_key_schedule_t *ks)
{
    if (!key || !ks)
        return AES_ERR_NULL;
    if (key_bytes != 16 && key_bytes != 24 && key_bytes != 32)
        return AES_ERR_KEYLEN;
    expand_schedule(key, (uint32_t)key_bytes, ks, kTables.sbox);
    return AES_OK;
}

}  // namespace aesmi

using namespace aesmi;

namespace {

bool aligned16(const void *p)
{
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
}

// in == out is fine; any other intersection of [in, in+n) and [out, out+n) is not.
bool bad_overlap(const void *in, const void *out, size_t n)
{
    uintptr_t a = reinterpret_cast<uintptr_t>(in), b = reinterpret_cast<uintptr_t>(out);
    if (a == b)
        return false;
    return a < b + n && b < a + n;
}

aes_status_t from_hip(hipError_t e)
{
    return e == hipSuccess ? AES_OK : AES_ERR_HIP;
}

uint32_t layout_of(const aes_launch_t *launch)
{
    return launch ? launch->layout : (uint32_t)AES_LAYOUT_AUTO;
}

bool valid_batch_tune(const aes_batch_tune_t *tune)
{
    if (!tune)
        return true;
    if (tune->layout > AES_LAYOUT_BITSLICE)
        return false;
    if (tune->wg_size && (tune->wg_size % 64 || tune->wg_size > 1024))
        return false;
    if (tune->grid_per_cu > 64)
        return false;
    if (tune->tile_blocks && (tune->tile_blocks % 64 || tune->tile_blocks > (1u << 20)))
        return false;
    if (tune->blocks_per_lane && tune->blocks_per_lane != 1 && tune->blocks_per_lane != 2 &&
        tune->blocks_per_lane != 4)
        return false;
    if (tune->layout == AES_LAYOUT_BITSLICE &&
        (tune->wg_size > 256 || (tune->tile_blocks && tune->tile_blocks % 2048)))
        return false;
    return true;
}

bool valid_launch(const aes_launch_t *launch)
{
    if (!launch)
        return true;
    if (launch->layout > AES_LAYOUT_BITSLICE)
        return false;
    if (launch->wg_size && (launch->wg_size % 64 || launch->wg_size > 1024))
        return false;
    if (launch->blocks_per_lane && launch->blocks_per_lane != 1 &&
        launch->blocks_per_lane != 2 && launch->blocks_per_lane != 4)
        return false;
    if (launch->grid_per_cu > 64)
        return false;
    if (launch->ctr_precompute > 2)
        return false;
    // the bitsliced kernels run workgroups of at most 256 threads
    if (launch->layout == AES_LAYOUT_BITSLICE && launch->wg_size > 256)
        return false;
    return true;
}

aes_status_t ecb_common(bool decrypt, const aes_key_schedule_t *ks, const void *in, void *out,
                        size_t nbytes, const aes_launch_t *launch, void *stream)
{
    if (nbytes == 0)
        return AES_OK;
    if (!ks || !in || !out)
        return AES_ERR_NULL;
    if (nbytes % 16)
        return AES_ERR_LENGTH;
    if (!aligned16(in) || !aligned16(out))
        return AES_ERR_ALIGN;
    if (bad_overlap(in, out, nbytes))
        return AES_ERR_OVERLAP;
    if (!valid_launch(launch))
        return AES_ERR_CONFIG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (layout_of(launch) == AES_LAYOUT_BITSLICE)
        return from_hip(bitslice_ecb(decrypt, ks, in, out, nbytes / 16, launch, s));
    return from_hip(ttable_ecb(decrypt, ks, in, out, nbytes / 16, launch, s));
}

}  // namespace

extern "C" {

aes_status_t aes_expand_key(const uint8_t *key, size_t key_bytes, aes_key_schedule_t *ks_host)
{
    return expand_key_host(key, key_bytes, ks_host);
}

aes_status_t aes_expand_keys_device(const uint8_t *keys_dev, size_t key_bytes, size_t nkeys,
                                    aes_key_schedule_t *ks_dev, void *stream)
{
    if (key_bytes != 16 && key_bytes != 24 && key_bytes != 32)
        return AES_ERR_KEYLEN;
    if (nkeys == 0)
        return AES_OK;
    if (!keys_dev || !ks_dev)
        return AES_ERR_NULL;
    return from_hip(expand_keys_device(keys_dev, (uint32_t)key_bytes, nkeys, ks_dev,
                                       static_cast<hipStream_t>(stream)));
}

aes_status_t aes_ecb_encrypt(const aes_key_schedule_t *ks_dev, const void *in_dev,
                             void *out_dev, size_t nbytes, void *stream)
{
    return ecb_common(false, ks_dev, in_dev, out_dev, nbytes, nullptr, stream);
}

aes_status_t aes_ecb_decrypt(const aes_key_schedule_t *ks_dev, const void *in_dev,
                             void *out_dev, size_t nbytes, void *stream)
{
    return ecb_common(true, ks_dev, in_dev, out_dev, nbytes, nullptr, stream);
}

aes_status_t aes_ecb_encrypt_ex(const aes_key_schedule_t *ks_dev, const void *in_dev,
                                void *out_dev, size_t nbytes, const aes_launch_t *launch,
                                void *stream)
{
    return ecb_common(false, ks_dev, in_dev, out_dev, nbytes, launch, stream);
}

aes_status_t aes_ecb_decrypt_ex(const aes_key_schedule_t *ks_dev, const void *in_dev,
                                void *out_dev, size_t nbytes, const aes_launch_t *launch,
                                void *stream)
{
    return ecb_common(true, ks_dev, in_dev, out_dev, nbytes, launch, stream);
}

aes_status_t aes_ctr_xcrypt_ex(const aes_key_schedule_t *ks_dev, const uint8_t *nonce,
                               uint32_t ctr0, const void *in_dev, void *out_dev, size_t nbytes,
                               const aes_launch_t *launch, void *stream)
{
    if (nbytes == 0)
        return AES_OK;
    if (!ks_dev || !nonce || !in_dev || !out_dev)
        return AES_ERR_NULL;
    if (!aligned16(in_dev) || !aligned16(out_dev))
        return AES_ERR_ALIGN;
    if (bad_overlap(in_dev, out_dev, nbytes))
        return AES_ERR_OVERLAP;
    const uint64_t nblocks = ((uint64_t)nbytes + 15u) / 16u;
    if ((uint64_t)ctr0 + nblocks > (1ull << 32))
        return AES_ERR_COUNTER;
    if (!valid_launch(launch))
        return AES_ERR_CONFIG;
    uint32_t nw[3];
    for (int c = 0; c < 3; ++c)
        nw[c] = (uint32_t)nonce[4 * c] | ((uint32_t)nonce[4 * c + 1] << 8) |
                ((uint32_t)nonce[4 * c + 2] << 16) | ((uint32_t)nonce[4 * c + 3] << 24);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (layout_of(launch) == AES_LAYOUT_BITSLICE)
        return from_hip(bitslice_ctr(ks_dev, nw, ctr0, in_dev, out_dev, nbytes, launch, s));
    return from_hip(ttable_ctr(ks_dev, nw, ctr0, in_dev, out_dev, nbytes, launch, s));
}

aes_status_t aes_ctr_xcrypt(const aes_key_schedule_t *ks_dev, const uint8_t *nonce,
                            uint32_t ctr0, const void *in_dev, void *out_dev, size_t nbytes,
                            void *stream)
{
    return aes_ctr_xcrypt_ex(ks_dev, nonce, ctr0, in_dev, out_dev, nbytes, nullptr, stream);
}

static aes_status_t cbc_common(bool decrypt, const aes_key_schedule_t *ks, const void *iv,
                               size_t iv_stride, const void *in, void *out, size_t nmsg,
                               size_t msg_bytes, void *stream)
{
    if (nmsg == 0 || msg_bytes == 0)
        return AES_OK;
    if (!ks || !iv || !in || !out)
        return AES_ERR_NULL;
    if (msg_bytes % 16)
        return AES_ERR_LENGTH;
    if (iv_stride != 0 && iv_stride != 16)
        return AES_ERR_CONFIG;
    if (!aligned16(in) || !aligned16(out) || !aligned16(iv))
        return AES_ERR_ALIGN;
    if (nmsg > SIZE_MAX / msg_bytes)
        return AES_ERR_LENGTH;
    const size_t nbytes = nmsg * msg_bytes;
    if (decrypt ? (in == out || bad_overlap(in, out, nbytes)) : bad_overlap(in, out, nbytes))
        return AES_ERR_OVERLAP;
    return from_hip(cbc(decrypt, ks, iv, iv_stride ? 1u : 0u, in, out, nmsg, msg_bytes / 16,
                        static_cast<hipStream_t>(stream)));
}

aes_status_t aes_cbc_encrypt(const aes_key_schedule_t *ks_dev, const void *iv_dev,
                             size_t iv_stride, const void *in_dev, void *out_dev, size_t nmsg,
                             size_t msg_bytes, void *stream)
{
    return cbc_common(false, ks_dev, iv_dev, iv_stride, in_dev, out_dev, nmsg, msg_bytes, stream);
}

aes_status_t aes_cbc_decrypt(const aes_key_schedule_t *ks_dev, const void *iv_dev,
                             size_t iv_stride, const void *in_dev, void *out_dev, size_t nmsg,
                             size_t msg_bytes, void *stream)
{
    return cbc_common(true, ks_dev, iv_dev, iv_stride, in_dev, out_dev, nmsg, msg_bytes, stream);
}

static bool aligned256(const void *p)
{
    return (reinterpret_cast<uintptr_t>(p) & 255u) == 0;
}

static uint32_t le_word(const uint8_t *b)
{
    return (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) |
           ((uint32_t)b[3] << 24);
}

size_t aes_gcm_workspace_bytes(size_t aad_len, size_t nbytes)
{
    return gcm_workspace_bytes(aad_len, nbytes);
}

static aes_status_t gcm_common(bool decrypt, const aes_key_schedule_t *ks, const uint8_t *iv,
                               const void *aad, size_t aad_len, const void *in, void *out,
                               size_t nbytes, void *tag, void *ws, size_t ws_bytes, void *stream)
{
    if (!ks || !iv || !tag || !ws || (nbytes && (!in || !out)) || (aad_len && !aad))
        return AES_ERR_NULL;
    if (aad_len >= (1ull << 61))
        return AES_ERR_LENGTH;
    if (!aligned16(tag) || !aligned256(ws) || (nbytes && (!aligned16(in) || !aligned16(out))) ||
        (aad_len && !aligned16(aad)))
        return AES_ERR_ALIGN;
    if (nbytes && bad_overlap(in, out, nbytes))
        return AES_ERR_OVERLAP;
    // counter blocks 2 .. 2 + ceil(n / 16) - 1 must not wrap (SP 800-38D sec. 5.2.1.1)
    if (((uint64_t)nbytes + 15u) / 16u + 2u > (1ull << 32))
        return AES_ERR_COUNTER;
    if (ws_bytes < gcm_workspace_bytes(aad_len, nbytes))
        return AES_ERR_CONFIG;
    const uint32_t ivw[3] = {le_word(iv), le_word(iv + 4), le_word(iv + 8)};
    return from_hip(gcm(decrypt, ks, ivw, aad, aad_len, in, out, nbytes, tag, ws,
                        static_cast<hipStream_t>(stream)));
}

aes_status_t aes_gcm_encrypt(const aes_key_schedule_t *ks_dev, const uint8_t *iv,
                             const void *aad_dev, size_t aad_len, const void *in_dev,
                             void *out_dev, size_t nbytes, void *tag_dev, void *ws_dev,
                             size_t ws_bytes, void *stream)
{
    return gcm_common(false, ks_dev, iv, aad_dev, aad_len, in_dev, out_dev, nbytes, tag_dev,
                      ws_dev, ws_bytes, stream);
}

aes_status_t aes_gcm_decrypt(const aes_key_schedule_t *ks_dev, const uint8_t *iv,
                             const void *aad_dev, size_t aad_len, const void *in_dev,
                             void *out_dev, size_t nbytes, void *tag_dev, void *ws_dev,
                             size_t ws_bytes, void *stream)
{
    return gcm_common(true, ks_dev, iv, aad_dev, aad_len, in_dev, out_dev, nbytes, tag_dev,
                      ws_dev, ws_bytes, stream);
}

size_t aes_ghash_workspace_bytes(size_t nblocks)
{
    return ghash_workspace_bytes(nblocks);
}

aes_status_t aes_ghash(const uint8_t *h, const void *x_dev, size_t nblocks, void *y_dev,
                       void *ws_dev, size_t ws_bytes, void *stream)
{
    if (!h || !y_dev || !ws_dev || (nblocks && !x_dev))
        return AES_ERR_NULL;
    if (!aligned16(y_dev) || !aligned256(ws_dev) || (nblocks && !aligned16(x_dev)))
        return AES_ERR_ALIGN;
    if (nblocks > (1ull << 40))
        return AES_ERR_LENGTH;
    if (ws_bytes < ghash_workspace_bytes(nblocks))
        return AES_ERR_CONFIG;
    const uint32_t hw[4] = {le_word(h), le_word(h + 4), le_word(h + 8), le_word(h + 12)};
    return from_hip(ghash(hw, x_dev, nblocks, y_dev, ws_dev, static_cast<hipStream_t>(stream)));
}

size_t aes_batched_workspace_bytes(uint32_t nsegs)
{
    return batched_workspace_bytes(nsegs);
}

aes_status_t aes_ctr_xcrypt_batched(const aes_segment_t *segs_dev, uint32_t nsegs,
                                    const aes_key_schedule_t *ks_table_dev, uint32_t nkeys,
                                    const uint8_t *in_base_dev, uint8_t *out_base_dev,
                                    const aes_batch_tune_t *tune, void *ws_dev, size_t ws_bytes,
                                    void *stream)
{
    if (nsegs == 0)
        return AES_OK;
    if (!segs_dev || !ks_table_dev || !in_base_dev || !out_base_dev || !ws_dev)
        return AES_ERR_NULL;
    if (nkeys == 0)
        return AES_ERR_SEGMENT;
    if (!aligned16(in_base_dev) || !aligned16(out_base_dev) || !aligned16(segs_dev) ||
        (reinterpret_cast<uintptr_t>(ws_dev) & 255u))
        return AES_ERR_ALIGN;
    if (ws_bytes < batched_workspace_bytes(nsegs))
        return AES_ERR_CONFIG;
    if (!valid_batch_tune(tune))
        return AES_ERR_CONFIG;
    return from_hip(batched_ctr(segs_dev, nsegs, ks_table_dev, nkeys, in_base_dev,
                                out_base_dev, tune, ws_dev, static_cast<hipStream_t>(stream)));
}

aes_status_t aes_batched_read_status(const void *ws_dev, void *stream, int32_t *status_out)
{
    if (!ws_dev || !status_out)
        return AES_ERR_NULL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t v = 0;
    hipError_t e = hipMemcpyAsync(&v, ws_dev, sizeof(v), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return AES_ERR_HIP;
    *status_out = v;
    return AES_OK;
}

aes_status_t aes_ctr_xcrypt_batched_noalloc(const aes_segment_t *segs_dev, uint32_t nsegs,
                                            const aes_key_schedule_t *ks_table_dev,
                                            uint32_t nkeys, const uint8_t *in_base_dev,
                                            uint8_t *out_base_dev, const aes_batch_tune_t *tune,
                                            int32_t *status_dev, void *stream)
{
    if (nsegs == 0)
        return AES_OK;
    if (!segs_dev || !ks_table_dev || !in_base_dev || !out_base_dev)
        return AES_ERR_NULL;
    if (nkeys == 0)
        return AES_ERR_SEGMENT;
    if (!aligned16(in_base_dev) || !aligned16(out_base_dev) || !aligned16(segs_dev) ||
        (reinterpret_cast<uintptr_t>(status_dev) & 3u))
        return AES_ERR_ALIGN;
    if (nsegs > batched_noalloc_max_segs() || !valid_batch_tune(tune))
        return AES_ERR_CONFIG;
    return from_hip(batched_ctr_noalloc(segs_dev, nsegs, ks_table_dev, nkeys, in_base_dev,
                                        out_base_dev, tune, status_dev,
                                        static_cast<hipStream_t>(stream)));
}

struct aes_batched_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

aes_status_t aes_batched_graph_create(const aes_segment_t *segs_dev, uint32_t nsegs,
                                      const aes_key_schedule_t *ks_table_dev, uint32_t nkeys,
                                      const uint8_t *in_base_dev, uint8_t *out_base_dev,
                                      const aes_batch_tune_t *tune, void *ws_dev,
                                      size_t ws_bytes, void *stream,
                                      aes_batched_graph_t **graph_out)
{
    if (!graph_out)
        return AES_ERR_NULL;
    *graph_out = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStream_t cap = s;
    bool own = false;
    if (!s) {
        // The null stream cannot be captured: record on a private stream.
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
            return AES_ERR_HIP;
        own = true;
    }
    hipGraph_t g = nullptr;
    aes_status_t st = AES_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = AES_ERR_HIP;
    } else {
        st = aes_ctr_xcrypt_batched(segs_dev, nsegs, ks_table_dev, nkeys, in_base_dev,
                                    out_base_dev, tune, ws_dev, ws_bytes, cap);
        hipError_t e = hipStreamEndCapture(cap, &g);
        if (st == AES_OK && e != hipSuccess)
            st = AES_ERR_HIP;
    }
    if (own)
        (void)hipStreamDestroy(cap);
    if (st != AES_OK) {
        if (g)
            (void)hipGraphDestroy(g);
        return st;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return AES_ERR_HIP;
    }
    aes_batched_graph_t *obj = new (std::nothrow) aes_batched_graph_t{g, ex};
    if (!obj) {
        (void)hipGraphExecDestroy(ex);
        (void)hipGraphDestroy(g);
        return AES_ERR_HIP;
    }
    *graph_out = obj;
    return AES_OK;
}

aes_status_t aes_batched_graph_launch(aes_batched_graph_t *graph, void *stream)
{
    if (!graph)
        return AES_ERR_NULL;
    return from_hip(hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)));
}

aes_status_t aes_batched_graph_destroy(aes_batched_graph_t *graph)
{
    if (!graph)
        return AES_OK;
    hipError_t e1 = hipGraphExecDestroy(graph->exec);
    hipError_t e2 = hipGraphDestroy(graph->graph);
    delete graph;
    return (e1 == hipSuccess && e2 == hipSuccess) ? AES_OK : AES_ERR_HIP;
}

static aes_status_t check_serve_setup(const uint8_t *keys32, const uint8_t *key_len,
                                      size_t nkeys, const aes_serve_params_t *params)
{
    if (!keys32 || !key_len || !params)
        return AES_ERR_NULL;
    const aes_serve_params_t &pr = *params;
    if (pr.nslots == 0 || pr.nstreams == 0 || pr.nstreams > kServeMaxStreams ||
        pr.max_batch_reqs == 0 || pr.max_batch_reqs > kServeMaxBatch || pr.hbm_budget == 0 ||
        pr.max_batch_bytes == 0 || !(pr.window_s >= 0.0) || pr.window_s > 1e9 ||
        pr.realtime > 1)
        return AES_ERR_CONFIG;
    for (size_t i = 0; i < nkeys; ++i)
        if (key_len[i] != 16 && key_len[i] != 24 && key_len[i] != 32)
            return AES_ERR_KEYLEN;
    return AES_OK;
}

static aes_status_t check_serve_trace(const aes_serve_request_t *reqs, size_t nreq, size_t nkeys,
                                      const void *pool_dev, size_t pool_bytes, void *out_dev,
                                      size_t out_bytes, double *latency_s, uint64_t *out_off)
{
    if (!reqs || !pool_dev || !out_dev || !latency_s || !out_off)
        return AES_ERR_NULL;
    if (!aligned16(pool_dev) || !aligned16(out_dev))
        return AES_ERR_ALIGN;
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(pool_dev),
                    o0 = reinterpret_cast<uintptr_t>(out_dev);
    if (p0 < o0 + out_bytes && o0 < p0 + pool_bytes)
        return AES_ERR_OVERLAP;
    if (out_bytes < 16)
        return AES_ERR_CONFIG;
    for (size_t i = 0; i < nreq; ++i) {
        const aes_serve_request_t &r = reqs[i];
        if (r.in_off & 15u)
            return AES_ERR_ALIGN;
        const uint64_t nblk = (r.nbytes + 15u) / 16u;
        if (r.nbytes == 0 || r.key_id >= nkeys || r.reserved != 0 ||
            r.in_off > pool_bytes || r.nbytes > pool_bytes - r.in_off ||
            (uint64_t)r.ctr0 + nblk > (1ull << 32) || !(r.arrival_s >= 0.0) ||
            !(r.arrival_s < 1e18) || (i && r.arrival_s < reqs[i - 1].arrival_s))
            return AES_ERR_SEGMENT;
    }
    return AES_OK;
}

aes_status_t aes_server_create(const uint8_t *keys32, const uint8_t *key_len, size_t nkeys,
                               const aes_serve_params_t *params, aes_server_t **server_out)
{
    if (!server_out)
        return AES_ERR_NULL;
    *server_out = nullptr;
    const aes_status_t st = check_serve_setup(keys32, key_len, nkeys, params);
    if (st != AES_OK)
        return st;
    return server_create(*params, keys32, key_len, nkeys, server_out);
}

aes_status_t aes_server_run(aes_server_t *server, const aes_serve_request_t *reqs, size_t nreq,
                            const void *pool_dev, size_t pool_bytes, void *out_dev,
                            size_t out_bytes, double *latency_s, uint64_t *out_off,
                            aes_serve_stats_t *stats)
{
    if (stats)
        *stats = aes_serve_stats_t{};
    if (!server)
        return AES_ERR_NULL;
    if (nreq == 0)
        return AES_OK;
    const aes_status_t st = check_serve_trace(reqs, nreq, server_nkeys(server), pool_dev,
                                              pool_bytes, out_dev, out_bytes, latency_s, out_off);
    if (st != AES_OK)
        return st;
    return server_run(server, reqs, nreq, static_cast<const uint8_t *>(pool_dev),
                      static_cast<uint8_t *>(out_dev), out_bytes, latency_s, out_off, stats);
}

aes_status_t aes_server_destroy(aes_server_t *server)
{
    server_destroy(server);
    return AES_OK;
}

aes_status_t aes_serve_run(const aes_serve_request_t *reqs, size_t nreq, const uint8_t *keys32,
                           const uint8_t *key_len, size_t nkeys, const void *pool_dev,
                           size_t pool_bytes, void *out_dev, size_t out_bytes,
                           const aes_serve_params_t *params, double *latency_s,
                           uint64_t *out_off, aes_serve_stats_t *stats)
{
    if (stats)
        *stats = aes_serve_stats_t{};
    if (nreq == 0)
        return AES_OK;
    aes_status_t st = check_serve_setup(keys32, key_len, nkeys, params);
    if (st == AES_OK)
        st = check_serve_trace(reqs, nreq, nkeys, pool_dev, pool_bytes, out_dev, out_bytes,
                               latency_s, out_off);
    if (st != AES_OK)
        return st;
    aes_server_t *srv = nullptr;
    st = server_create(*params, keys32, key_len, nkeys, &srv);
    if (st != AES_OK)
        return st;
    st = server_run(srv, reqs, nreq, static_cast<const uint8_t *>(pool_dev),
                    static_cast<uint8_t *>(out_dev), out_bytes, latency_s, out_off, stats);
    server_destroy(srv);
    return st;
}

const char *aes_status_string(aes_status_t status)
{
    switch (status) {
    case AES_OK: return "ok";
    case AES_ERR_NULL: return "null pointer";
    case AES_ERR_KEYLEN: return "key length must be 16, 24 or 32 bytes";
    case AES_ERR_LENGTH: return "ECB length must be a multiple of 16 bytes";
    case AES_ERR_ALIGN: return "device pointer not 16-byte aligned";
    case AES_ERR_OVERLAP: return "input and output overlap without being equal";
    case AES_ERR_COUNTER: return "counter range exceeds 2^32 blocks";
    case AES_ERR_SEGMENT: return "invalid segment table entry";
    case AES_ERR_HIP: return "HIP runtime error";
    case AES_ERR_CONFIG: return "invalid launch configuration or workspace";
    case AES_ERR_DEVICE: return "no usable gfx950 device";
    }
    return "unknown status";
}

const char *aes_version(void)
{
    return "aesmi 0.1 (gfx950)";
}

int aes_device_cu_count(void)
{
    return device_cu_count();
}

}  // extern "C"
