// internal.hpp -- launchers shared between the translation units of libaesmi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aesmi.h"

namespace aesmi {

// Resolved launch shape of one kernel launch.
struct Shape {
    uint32_t wg;      // threads per workgroup
    uint32_t grid;    // workgroups
    uint32_t bpl;     // blocks per lane per loop iteration (1, 2 or 4)
};

// Compute units of the current device (cached per device; 0 if none).
int device_cu_count();

// --- T-table kernels (ttable.hip) ------------------------------------------
// Full 16-byte blocks only for ECB; CTR handles a ragged tail itself.
hipError_t ttable_ecb(bool decrypt, const aes_key_schedule_t *ks, const void *in,
                      void *out, uint64_t nblocks, const aes_launch_t *launch,
                      hipStream_t stream);
hipError_t ttable_ctr(const aes_key_schedule_t *ks, const uint32_t nonce_words[3],
                      uint32_t ctr0, const void *in, void *out, uint64_t nbytes,
                      const aes_launch_t *launch, hipStream_t stream);

// --- bitsliced kernels (bitslice.hip) --------------------------------------
hipError_t bitslice_ecb(bool decrypt, const aes_key_schedule_t *ks, const void *in,
                        void *out, uint64_t nblocks, const aes_launch_t *launch,
                        hipStream_t stream);
hipError_t bitslice_ctr(const aes_key_schedule_t *ks, const uint32_t nonce_words[3],
                        uint32_t ctr0, const void *in, void *out, uint64_t nbytes,
                        const aes_launch_t *launch, hipStream_t stream);

// --- CBC over a matrix of messages (cbc.hip) --------------------------------
hipError_t cbc(bool decrypt, const aes_key_schedule_t *ks, const void *iv, uint32_t iv_step,
               const void *in, void *out, uint64_t nmsg, uint64_t nblk, hipStream_t stream);

// --- Galois/Counter Mode and GHASH (gcm.hip) --------------------------------
size_t gcm_workspace_bytes(uint64_t aad_len, uint64_t nbytes);
size_t ghash_workspace_bytes(uint64_t nblocks);
hipError_t gcm(bool decrypt, const aes_key_schedule_t *ks, const uint32_t iv_words[3],
               const void *aad, uint64_t aad_len, const void *in, void *out, uint64_t nbytes,
               void *tag, void *ws, hipStream_t stream);
hipError_t ghash(const uint32_t h_words[4], const void *x, uint64_t nblocks, void *y, void *ws,
                 hipStream_t stream);

// --- device key expansion (keyexp.hip) -------------------------------------
hipError_t expand_keys_device(const uint8_t *keys, uint32_t key_bytes, uint64_t nkeys,
                              aes_key_schedule_t *ks, hipStream_t stream);
// Copy `bytes` (a multiple of 16) from pinned host memory src_host to dst_dev
// and expand nfill keys into table, in one launch on `stream`: key i is the
// first lens[i] bytes (16, 24 or 32) of keys32 + 32 i and goes to row
// slots[i] (keys32, lens and slots in mapped host memory); rows get nr,
// key_bytes and rk_enc, not rk_dec.
hipError_t stage_and_expand(const void *src_host, void *dst_dev, size_t bytes,
                            const uint8_t *keys32, const uint8_t *lens, const uint32_t *slots,
                            uint32_t nfill, aes_key_schedule_t *table, hipStream_t stream);

// --- serving loop (serve.hip); arguments checked in api.hip ----------------
constexpr uint32_t kServeMaxStreams = 8;
constexpr uint32_t kServeMaxBatch = 65536;
aes_status_t server_create(const aes_serve_params_t &pr, const uint8_t *keys32,
                           const uint8_t *key_len, size_t nkeys, aes_server_t **out);
aes_status_t server_run(aes_server_t *srv, const aes_serve_request_t *reqs, size_t nreq,
                        const uint8_t *pool, uint8_t *out, uint64_t out_bytes, double *latency_s,
                        uint64_t *out_off, aes_serve_stats_t *stats);
void server_destroy(aes_server_t *srv);
size_t server_nkeys(const aes_server_t *srv);

// --- batched persistent kernel (batched.hip) -------------------------------
size_t batched_workspace_bytes(uint32_t nsegs);
hipError_t batched_ctr(const aes_segment_t *segs, uint32_t nsegs,
                       const aes_key_schedule_t *ks_table, uint32_t nkeys,
                       const uint8_t *in_base, uint8_t *out_base,
                       const aes_batch_tune_t *tune, void *ws, hipStream_t stream);

// The prepare kernel's work done on the host, for callers that already hold
// the segment table in host memory and have checked it: writes the workspace
// header and tile_start[0..nsegs] into ws_host (batched_workspace_bytes(nsegs)
// bytes), to be copied to the device workspace before the launch.
void batched_prepare_host(const aes_segment_t *segs, uint32_t nsegs, uint32_t tile_blocks,
                          void *ws_host);
// The T-table persistent kernel alone (1,024 threads, one workgroup per CU)
// over a workspace that batched_prepare_host filled with the given tile size.
hipError_t batched_ctr_prepared(const aes_segment_t *segs, uint32_t nsegs,
                                const aes_key_schedule_t *ks_table, const uint8_t *in_base,
                                uint8_t *out_base, void *ws, hipStream_t stream);
// Default tiles of the batched kernels.  T-table, 10^4 messages of 1 B..1 MiB
// (1,024-thread workgroups, four blocks per lane): 256 / 512 / 1,024 / 2,048 /
// 4,096-block tiles 0.494 / 0.444 / 0.429 / 0.434 / 0.457 ms.  The bitsliced
// kernel works in batches of 2,048 blocks.
constexpr uint32_t kBatchedTileBlocks = 1024;
constexpr uint32_t kBatchedBitsliceTileBlocks = 2048;

// The batched call on the library's own static device workspace (no
// allocation); at most batched_noalloc_max_segs() segments.  When status is
// not NULL the segment status word is copied there after the launch.
uint32_t batched_noalloc_max_segs();
hipError_t batched_ctr_noalloc(const aes_segment_t *segs, uint32_t nsegs,
                               const aes_key_schedule_t *ks_table, uint32_t nkeys,
                               const uint8_t *in_base, uint8_t *out_base,
                               const aes_batch_tune_t *tune, int32_t *status, hipStream_t stream);

// Host key expansion into the public struct (api.hip).
aes_status_t expand_key_host(const uint8_t *key, size_t key_bytes, aes_key_schedule_t *ks);

}  // namespace aesmi
