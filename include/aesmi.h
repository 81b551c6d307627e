/*
 * aesmi.h -- C ABI of the MI355X (gfx950) AES library.
 *
 * The library encrypts very many independent 16-byte blocks on one GPU: the
 * AES cipher (key expansion; rounds of SubBytes, ShiftRows, MixColumns and
 * AddRoundKey, the last round without MixColumns) in ECB and counter (CTR)
 * mode, as framed algebraically in Kepner et al., arXiv 1506.08503 (sec. II,
 * App. A1-A5).  128-, 192- and 256-bit keys (10, 12, 14 rounds).  Also: the
 * paper's CBC over a matrix of messages (App. A1, A4), many messages with
 * their own keys in one launch (the per-row V and K of sec. II), and GCM
 * (NIST SP 800-38D) for authenticated encryption.
 *
 * Conventions shared by every entry point
 *  - Plain C types only.  Device buffers are raw device pointers; `stream` is
 *    a hipStream_t passed as void* (NULL = the null stream).
 *  - The caller owns every buffer.  No entry point allocates device memory,
 *    except that aes_batched_graph_create builds a HIP graph (set-up code),
 *    aes_serve_run sets up its key cache and staging for a whole run, and
 *    aes_server_create does the same once for many runs;
 *    aes_ctr_xcrypt_batched_noalloc works in a static workspace of the
 *    library's own instead of a caller's.
 *  - Launching entry points are stream-ordered and asynchronous: AES_OK means
 *    the arguments passed validation and the work was enqueued on `stream`.
 *    Argument errors are returned before any HIP call is made.
 *  - Device data buffers must be 16-byte aligned.  in == out (in place) is
 *    allowed; any other overlap of the input and output ranges is an error.
 *  - nbytes == 0 is a no-op that returns AES_OK (pointers are not checked).
 *  - Byte order: block k of a buffer is bytes [16k, 16k+16); byte j of a
 *    block is state row j % 4, column j / 4 (the order the paper's ShiftRows
 *    index vectors of App. A1 / A4 imply).
 */
#ifndef AESMI_H
#define AESMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AES_OK = 0,
    AES_ERR_NULL = -1,     /* a required pointer is NULL                        */
    AES_ERR_KEYLEN = -2,   /* key length not 16, 24 or 32 bytes                 */
    AES_ERR_LENGTH = -3,   /* ECB length not a multiple of 16                   */
    AES_ERR_ALIGN = -4,    /* a device data pointer is not 16-byte aligned      */
    AES_ERR_OVERLAP = -5,  /* input and output overlap without being equal      */
    AES_ERR_COUNTER = -6,  /* CTR: ctr0 + number of blocks exceeds 2^32         */
    AES_ERR_SEGMENT = -7,  /* batched: invalid segment table entry              */
    AES_ERR_HIP = -8,      /* the HIP runtime reported an error                 */
    AES_ERR_CONFIG = -9,   /* invalid launch configuration / workspace too small*/
    AES_ERR_DEVICE = -10   /* no usable gfx950 device                           */
} aes_status_t;

/*
 * Expanded key: the Nr + 1 round keys of the key schedule (App. A3 for 128-bit
 * keys; FIPS-197 sec. 5.2 for 192 / 256).  Round key r, column c is
 * rk_enc[4 r + c], a little-endian word whose byte j is state row j.
 * rk_dec holds the keys of the equivalent inverse cipher: rk_dec[4 r + c] is
 * column c of InvMixColumns(round key Nr - r) for 0 < r < Nr, and the plain
 * round keys Nr and 0 at r = 0 and r = Nr.  Plain old data (488 bytes); it is
 * valid in host or device memory and carries no pointers.
 */
typedef struct aes_key_schedule {
    uint32_t nr;          /* 10, 12 or 14                                 */
    uint32_t key_bytes;   /* 16, 24 or 32                                 */
    uint32_t rk_enc[60];
    uint32_t rk_dec[60];
} aes_key_schedule_t;

/* Kernel layout for the round function. */
typedef enum {
    AES_LAYOUT_AUTO = 0,      /* library default (the measured faster one)        */
    AES_LAYOUT_TTABLE = 1,    /* lookup tables replicated in LDS per lane group     */
    AES_LAYOUT_BITSLICE = 2   /* constant-time bitsliced: 32 blocks per lane word   */
} aes_layout_t;

/* Launch shape.  Zero fields take the library default. */
typedef struct aes_launch {
    uint32_t layout;          /* aes_layout_t                                    */
    uint32_t wg_size;         /* threads per workgroup (multiple of 64, <= 1024) */
    uint32_t grid_per_cu;     /* workgroups per compute unit, at most 64.  The
                                 default sizes the grid from the input: table
                                 layout, one per CU up to 16384 blocks per wave
                                 and more beyond; bitsliced, one 2048-block
                                 batch per wave (at most 64 per CU)          */
    uint32_t blocks_per_lane; /* 16-byte blocks a lane carries per iteration     */
    uint32_t ctr_precompute;  /* CTR with the table layout only (ignored elsewhere):
                                 0 = default: the round-1 terms of the nonce
                                     columns once per thread and, with four
                                     blocks per lane, round 2 per 256-counter
                                     group (16 (Nr - 2) table reads per block);
                                 1 = round-1 nonce terms only (16 Nr - 12);
                                 2 = none, every round from the counter block
                                     (16 Nr).  The output is the same.       */
} aes_launch_t;

/*
 * aes_expand_key -- host key expansion (App. A3; FIPS-197 sec. 5.2).
 *   key       host pointer, key_bytes bytes (16, 24 or 32)
 *   ks_host   host output; fully overwritten
 * Returns AES_ERR_NULL, AES_ERR_KEYLEN or AES_OK.  Pure host code, no GPU.
 */
aes_status_t aes_expand_key(const uint8_t *key, size_t key_bytes,
                            aes_key_schedule_t *ks_host);

/*
 * aes_expand_keys_device -- key expansion of nkeys keys on the GPU, one key
 * per lane (App. A3).  keys_dev: device, nkeys * key_bytes bytes, key i at
 * offset i * key_bytes.  ks_dev: device array of nkeys schedules (output).
 * Same validation as aes_expand_key; nkeys == 0 is a no-op.
 */
aes_status_t aes_expand_keys_device(const uint8_t *keys_dev, size_t key_bytes,
                                    size_t nkeys, aes_key_schedule_t *ks_dev,
                                    void *stream);

/*
 * aes_ecb_encrypt / aes_ecb_decrypt -- ECB (sec. II): each 16-byte block of
 * in_dev is enciphered (App. A1 round sequence without the chaining) or
 * deciphered (App. A4 without the chaining) on its own into out_dev.
 *   ks_dev   device pointer to one key schedule
 *   nbytes   multiple of 16, else AES_ERR_LENGTH
 * The _ex forms take a launch shape (NULL = default).
 */
aes_status_t aes_ecb_encrypt(const aes_key_schedule_t *ks_dev, const void *in_dev,
                             void *out_dev, size_t nbytes, void *stream);
aes_status_t aes_ecb_decrypt(const aes_key_schedule_t *ks_dev, const void *in_dev,
                             void *out_dev, size_t nbytes, void *stream);
aes_status_t aes_ecb_encrypt_ex(const aes_key_schedule_t *ks_dev, const void *in_dev,
                                void *out_dev, size_t nbytes,
                                const aes_launch_t *launch, void *stream);
aes_status_t aes_ecb_decrypt_ex(const aes_key_schedule_t *ks_dev, const void *in_dev,
                                void *out_dev, size_t nbytes,
                                const aes_launch_t *launch, void *stream);

/*
 * aes_ctr_xcrypt -- counter mode (not in the paper; the cipher of sec. II
 * applied to counter blocks): keystream block i is the encryption of
 * nonce[0..11] followed by the big-endian 32-bit value ctr0 + i, and
 * out = in XOR keystream.  A short last block uses the first nbytes % 16
 * keystream bytes.  The same call decrypts.
 *   nonce    HOST pointer to 12 bytes (copied into the launch)
 *   nbytes   any length; ctr0 + ceil(nbytes / 16) must be <= 2^32, else
 *            AES_ERR_COUNTER (the counter never wraps silently)
 */
aes_status_t aes_ctr_xcrypt(const aes_key_schedule_t *ks_dev, const uint8_t *nonce,
                            uint32_t ctr0, const void *in_dev, void *out_dev,
                            size_t nbytes, void *stream);
aes_status_t aes_ctr_xcrypt_ex(const aes_key_schedule_t *ks_dev, const uint8_t *nonce,
                               uint32_t ctr0, const void *in_dev, void *out_dev,
                               size_t nbytes, const aes_launch_t *launch,
                               void *stream);

/*
 * aes_cbc_encrypt / aes_cbc_decrypt -- CBC over a matrix of messages, the
 * mode of the paper's listings (App. A1 encryption, App. A4 decryption):
 * nmsg rows of msg_bytes bytes each, row-major and contiguous in in_dev /
 * out_dev.  Block i of row r is enciphered after XOR with ciphertext block
 * i-1 of the same row (the row's IV for i = 0); decryption XORs the
 * previous ciphertext block after the inverse cipher.  The paper zero-pads
 * rows to a whole number of blocks (App. A1); here the caller passes padded
 * rows: msg_bytes % 16 != 0 is AES_ERR_LENGTH.
 *   iv_dev     device; iv_stride 16: one 16-byte IV per row (the per-row V of
 *              sec. II), iv_stride 0: one IV shared by all rows (App. A1)
 * Encryption is parallel across rows only (serial along a row) and may run
 * in place; decryption is parallel across all blocks and must not run in
 * place (AES_ERR_OVERLAP if the ranges intersect).  nmsg == 0 or
 * msg_bytes == 0 is a no-op.
 */
aes_status_t aes_cbc_encrypt(const aes_key_schedule_t *ks_dev, const void *iv_dev,
                             size_t iv_stride, const void *in_dev, void *out_dev,
                             size_t nmsg, size_t msg_bytes, void *stream);
aes_status_t aes_cbc_decrypt(const aes_key_schedule_t *ks_dev, const void *iv_dev,
                             size_t iv_stride, const void *in_dev, void *out_dev,
                             size_t nmsg, size_t msg_bytes, void *stream);

/*
 * Galois/Counter Mode, NIST SP 800-38D, with 96-bit IVs.  The paper's modes
 * (CBC, App. A1; counter mode, sec. II) give confidentiality only; GCM adds a
 * 128-bit authentication tag over the ciphertext and additional data:
 *   C = CTR_K(counter blocks IV || 2, IV || 3, ...) applied to P,
 *   T = E_K(IV || 1) ^ GHASH_H(A || 0-pad || C || 0-pad || len64(A) || len64(C)),
 *   H = E_K(0^128), GHASH_H(X_1..X_m) = sum_i X_i H^(m-i+1) in GF(2^128) with
 *   x^128 + x^7 + x^2 + x + 1 (SP 800-38D sec. 6.3-7.1, bit order of sec. 6.3).
 *   iv          host, 12 bytes (other IV lengths are not supported)
 *   aad_dev     device, aad_len bytes of additional authenticated data
 *               (16-byte aligned; NULL allowed when aad_len == 0)
 *   in_dev/out_dev  device, nbytes each (any nbytes >= 0; in place allowed)
 *   tag_dev     device, 16 bytes (16-byte aligned): the full 128-bit tag
 *   ws_dev      device workspace of at least aes_gcm_workspace_bytes(aad_len,
 *               nbytes) bytes, 256-byte aligned, private to the call until the
 *               stream has passed it (holds H, E_K(J0), the powers of H and the
 *               partial GHASH sums).
 * aes_gcm_decrypt computes the tag over the ciphertext in_dev (before it
 * writes out_dev, so in place is fine) and deciphers; comparing that tag with
 * the received one is the caller's step: per SP 800-38D sec. 7.2 the plaintext
 * must not be released unless they are equal.  Errors: AES_ERR_NULL,
 * AES_ERR_ALIGN, AES_ERR_OVERLAP, AES_ERR_COUNTER (more than 2^32 - 2 blocks),
 * AES_ERR_LENGTH (aad_len >= 2^61), AES_ERR_CONFIG (workspace too small).
 */
size_t aes_gcm_workspace_bytes(size_t aad_len, size_t nbytes);
aes_status_t aes_gcm_encrypt(const aes_key_schedule_t *ks_dev, const uint8_t *iv,
                             const void *aad_dev, size_t aad_len, const void *in_dev,
                             void *out_dev, size_t nbytes, void *tag_dev, void *ws_dev,
                             size_t ws_bytes, void *stream);
aes_status_t aes_gcm_decrypt(const aes_key_schedule_t *ks_dev, const uint8_t *iv,
                             const void *aad_dev, size_t aad_len, const void *in_dev,
                             void *out_dev, size_t nbytes, void *tag_dev, void *ws_dev,
                             size_t ws_bytes, void *stream);

/*
 * aes_ghash -- GHASH_H over nblocks 16-byte blocks (SP 800-38D Algorithm 2),
 * the authentication half of GCM on its own.
 *   h        host, 16 bytes: the hash subkey H
 *   x_dev    device, nblocks * 16 bytes (16-byte aligned)
 *   y_dev    device, 16 bytes (16-byte aligned): the result (zero if nblocks == 0)
 *   ws_dev   device workspace of aes_ghash_workspace_bytes(nblocks) bytes,
 *            256-byte aligned.
 */
size_t aes_ghash_workspace_bytes(size_t nblocks);
aes_status_t aes_ghash(const uint8_t *h, const void *x_dev, size_t nblocks, void *y_dev,
                       void *ws_dev, size_t ws_bytes, void *stream);

/*
 * Batched CTR: many messages, each with its own key schedule, nonce and
 * counter, in one persistent launch (the per-row V and K of sec. II applied to
 * messages of uneven length).  Message s reads nbytes bytes at
 * in_base + in_off and writes them at out_base + out_off, exactly as
 * aes_ctr_xcrypt would with ks_table[key_slot], its nonce and ctr0.
 */
typedef struct aes_segment {
    uint64_t in_off;      /* byte offset of the message in in_base (16-aligned)  */
    uint64_t out_off;     /* byte offset in out_base (16-aligned)                */
    uint64_t nbytes;      /* message length, any value >= 0                      */
    uint32_t key_slot;    /* index into ks_table                                  */
    uint32_t ctr0;        /* first counter value                                  */
    uint8_t  nonce[12];
    uint32_t reserved;    /* must be 0                                            */
} aes_segment_t;          /* 48 bytes */

/* Tuning of the batched launch.  Zero fields take the library default. */
typedef struct aes_batch_tune {
    uint32_t layout;          /* aes_layout_t                                  */
    uint32_t wg_size;         /* threads per workgroup                         */
    uint32_t grid_per_cu;     /* persistent workgroups per compute unit        */
    uint32_t tile_blocks;     /* 16-byte blocks per tile claimed by a wave     */
    uint32_t blocks_per_lane; /* table layout: 1, 2 or 4 blocks a lane carries
                                 at once (default 4, which also enables the
                                 round-1/2 precomputation over 256-counter
                                 groups); the bitsliced layout always packs
                                 32 blocks per lane and ignores it          */
} aes_batch_tune_t;

/*
 * Workspace the batched call needs (device bytes, 256-byte aligned by the
 * caller) for nsegs segments: the per-segment tile prefix sums, the tile
 * counter and the device status word.
 */
size_t aes_batched_workspace_bytes(uint32_t nsegs);

/*
 * aes_ctr_xcrypt_batched -- one persistent launch over a device segment table.
 *   segs_dev    device array of nsegs segments
 *   nkeys       number of schedules in ks_table_dev (key_slot must be < nkeys)
 *   ws_dev      device workspace of at least aes_batched_workspace_bytes(nsegs)
 *   tune        host pointer or NULL
 * Segment errors (bad slot, misaligned offset, counter overflow, reserved != 0,
 * a key schedule without a valid round count) are found on the device: that
 * segment is skipped and the status word in the workspace becomes
 * AES_ERR_SEGMENT; read it after the stream completes with
 * aes_batched_read_status.  Messages must not overlap each other's output.
 * Host-side errors, returned before any launch: AES_ERR_NULL (a NULL
 * pointer), AES_ERR_SEGMENT (nkeys == 0), AES_ERR_ALIGN (segs_dev or a base
 * pointer not 16-byte aligned, ws_dev not 256-byte aligned), AES_ERR_CONFIG
 * (workspace too small, or a tune field out of range: layout, wg_size a
 * multiple of 64 up to 1024 (256 bitsliced), grid_per_cu up to 64,
 * tile_blocks a multiple of 64 up to 2^20 (of 2048 bitsliced),
 * blocks_per_lane 0, 1, 2 or 4).  nsegs == 0
 * is a no-op that leaves the workspace untouched.
 */
aes_status_t aes_ctr_xcrypt_batched(const aes_segment_t *segs_dev, uint32_t nsegs,
                                    const aes_key_schedule_t *ks_table_dev,
                                    uint32_t nkeys, const uint8_t *in_base_dev,
                                    uint8_t *out_base_dev, const aes_batch_tune_t *tune,
                                    void *ws_dev, size_t ws_bytes, void *stream);

/* Status word of the last batched call that used ws_dev (synchronous copy on
 * `stream`; call after the batched launch). */
aes_status_t aes_batched_read_status(const void *ws_dev, void *stream,
                                     int32_t *status_out);

/*
 * aes_ctr_xcrypt_batched_noalloc -- aes_ctr_xcrypt_batched without a caller
 * workspace, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid allocation).  The
 * workspace is a static array inside the library, one per device, of fixed
 * size: nsegs may be at most 65,536.  The call allocates nothing (no
 * hipMalloc, no pinned memory, no library routine that allocates).
 *   status_dev  device int32 (4-byte aligned) that receives the segment
 *               status word (AES_OK or AES_ERR_SEGMENT) once the launch has
 *               run, or NULL when the caller does not want it
 * Other arguments, results and errors as aes_ctr_xcrypt_batched, plus
 * AES_ERR_CONFIG for nsegs > 65,536.  Every call on one device shares that
 * device's static workspace and keeps it after the call: calls that overlap
 * on one device (on different streams, or from different threads without
 * ordering) race and must not be issued; calls ordered on one stream are
 * fine.  nsegs == 0 is a no-op that leaves *status_dev untouched.
 */
aes_status_t aes_ctr_xcrypt_batched_noalloc(const aes_segment_t *segs_dev, uint32_t nsegs,
                                            const aes_key_schedule_t *ks_table_dev,
                                            uint32_t nkeys, const uint8_t *in_base_dev,
                                            uint8_t *out_base_dev,
                                            const aes_batch_tune_t *tune, int32_t *status_dev,
                                            void *stream);

/*
 * Graph form of the batched call: captures aes_ctr_xcrypt_batched with fixed
 * pointers into a HIP graph.  The caller may rewrite the contents of segs_dev,
 * the input and the key table between launches (nsegs is fixed per graph).
 *   aes_batched_graph_create  validates the arguments as the batched call
 *       does (its error codes), records the two kernels on `stream` (on a
 *       private stream if `stream` is NULL, which cannot be captured) and
 *       instantiates the graph.  It allocates: the handle in host memory and
 *       the executable graph inside the HIP runtime, so it is set-up code,
 *       not hot-path code.  *graph_out is NULL unless AES_OK is returned; the
 *       caller owns the handle and releases it with aes_batched_graph_destroy.
 *   aes_batched_graph_launch  enqueues the graph on `stream` (AES_ERR_NULL for
 *       a NULL handle, AES_ERR_HIP if the runtime refuses).
 *   aes_batched_graph_destroy releases the graph and the handle; NULL is a
 *       no-op.  Launches already enqueued must have completed.
 */
typedef struct aes_batched_graph aes_batched_graph_t;
aes_status_t aes_batched_graph_create(const aes_segment_t *segs_dev, uint32_t nsegs,
                                      const aes_key_schedule_t *ks_table_dev,
                                      uint32_t nkeys, const uint8_t *in_base_dev,
                                      uint8_t *out_base_dev,
                                      const aes_batch_tune_t *tune, void *ws_dev,
                                      size_t ws_bytes, void *stream,
                                      aes_batched_graph_t **graph_out);
aes_status_t aes_batched_graph_launch(aes_batched_graph_t *graph, void *stream);
aes_status_t aes_batched_graph_destroy(aes_batched_graph_t *graph);

/*
 * Serving: a continuous-batching request loop on the host that encrypts a
 * trace of CTR requests on the device (the per-row V and K of sec. II, as
 * requests arrive).  aes_serve_run plays the whole trace and returns when
 * every request is done or rejected:
 *  - requests are admitted in arrival order while the input plus output
 *    bytes of admitted, unfinished requests fit hbm_budget and their outputs
 *    fit the free part of the output area; a request whose input plus output
 *    exceeds the whole budget, or whose output exceeds the whole output
 *    area, is rejected;
 *  - the output area is a ring: a batch's outputs take one contiguous range
 *    of it, and the range is reused after the batch has completed and been
 *    handed to the consumer (on_batch), so admission waits on output memory
 *    that really frees;
 *  - key schedules live in a device cache of nslots rows (LRU among rows no
 *    in-flight batch uses, empty rows first); one batch takes at most
 *    nslots / nstreams of the free rows, so batches can overlap;
 *  - a batch closes when one of nstreams launch slots is free and nothing
 *    runs, or the queued bytes reach max_batch_bytes, or the oldest queued
 *    request has waited window_s, or the whole trace has arrived.  On the
 *    batch's stream one staging kernel copies its segment and tile tables
 *    (written on the host into mapped pinned memory) to the device and
 *    expands its missed keys into their rows, then aes_ctr_xcrypt_batched's
 *    T-table kernel runs it (tiles of 256 to 1,024 blocks by batch size);
 *    batches on different streams overlap;
 *  - a request's result is the CTR encryption of its payload with its key,
 *    nonce and ctr0, exactly as aes_ctr_xcrypt would give it alone.
 */
typedef struct aes_serve_request {
    double arrival_s;     /* scheduled arrival, seconds from the start         */
    uint64_t in_off;      /* payload offset in the input pool (16-aligned)     */
    uint64_t nbytes;      /* payload length (> 0)                              */
    uint32_t key_id;      /* index into the key set                            */
    uint32_t ctr0;        /* first counter value                               */
    uint8_t  nonce[12];
    uint32_t reserved;    /* must be 0                                         */
} aes_serve_request_t;    /* 48 bytes; requests sorted by arrival_s            */

/* Called on the thread that runs aes_serve_run once a batch has completed on
 * the device, with the batch's requests [first, first + count) (in request
 * order, contiguous).  Their outputs are at out_dev + out_off[i] and stay
 * there until the callback returns; after that the range may be reused.  The
 * callback may read or copy them (synchronously: anything it enqueues must be
 * complete before it returns) and must not call aes_serve_run. */
typedef void (*aes_serve_batch_fn)(void *user, uint64_t first, uint64_t count);

typedef struct aes_serve_params {
    uint32_t nslots;          /* key-schedule cache rows, >= 1                 */
    uint32_t nstreams;        /* batches in flight, 1 .. 8                     */
    uint32_t max_batch_reqs;  /* requests per batch, 1 .. 65536                */
    uint32_t realtime;        /* 1: requests arrive at arrival_s; 0: at once   */
    uint64_t hbm_budget;      /* admission budget in bytes (any value >= 1)    */
    uint64_t max_batch_bytes; /* payload bytes that close a batch (>= 1)       */
    double   window_s;        /* longest wait of the oldest queued request     */
    aes_serve_batch_fn on_batch;  /* consumer of completed batches, or NULL    */
    void    *user;            /* passed to on_batch                            */
} aes_serve_params_t;

typedef struct aes_serve_stats {
    uint64_t completed, rejected, batches, bytes;
    uint64_t key_hits, key_misses;   /* per request                            */
    uint64_t max_held;               /* peak admitted input + output bytes     */
    uint64_t max_out_used;           /* peak bytes of the output area in use   */
    uint32_t max_inflight;
    uint32_t reserved;
    double   elapsed_s;
} aes_serve_stats_t;

/*
 * aes_serve_run -- play a request trace (see above).
 *   reqs        host, nreq requests sorted by arrival_s
 *   keys32      host, nkeys x 32 bytes: key i in its first key_len[i] bytes
 *   key_len     host, nkeys bytes: 16, 24 or 32
 *   pool_dev    device input pool of pool_bytes bytes (16-byte aligned)
 *   out_dev     device output area of out_bytes bytes (16-byte aligned,
 *               at least 16), used as a ring: request i's output (padded to
 *               16 bytes) is written at out_dev + out_off[i]; with out_bytes
 *               at least the sum of all padded outputs nothing is reused and
 *               every output is still there after the call, otherwise a
 *               result is only guaranteed until on_batch returns for it
 *   latency_s   host out, nreq: completion minus scheduled arrival (seconds;
 *               +inf for a rejected request)
 *   out_off     host out, nreq: offset of the request's output in out_dev
 *               (UINT64_MAX when rejected)
 *   stats       host out, may be NULL
 * Every request and parameter is checked before the run starts: AES_ERR_NULL,
 * AES_ERR_KEYLEN (a key_len not 16/24/32), AES_ERR_ALIGN (pool, output or an
 * in_off not 16-aligned), AES_ERR_SEGMENT (a payload outside the pool, a
 * key_id >= nkeys, nbytes == 0, reserved != 0, ctr0 + blocks > 2^32, or
 * arrivals out of order), AES_ERR_OVERLAP (pool and output area intersect),
 * AES_ERR_CONFIG (parameters out of range, out_bytes < 16); AES_ERR_HIP if a
 * HIP call fails during the run (outputs and latencies are then incomplete).
 * Unlike the other entry points this one allocates: the device key table,
 * per-stream pinned and device staging, streams and events (set up before
 * the clock starts, freed before it returns).  Blocks the calling thread for
 * the whole run, polling the device; uses the current device.  The pool must
 * not be written while the call runs.
 */
aes_status_t aes_serve_run(const aes_serve_request_t *reqs, size_t nreq, const uint8_t *keys32,
                           const uint8_t *key_len, size_t nkeys, const void *pool_dev,
                           size_t pool_bytes, void *out_dev, size_t out_bytes,
                           const aes_serve_params_t *params, double *latency_s,
                           uint64_t *out_off, aes_serve_stats_t *stats);

/*
 * A server: the same loop with its set-up done once.  aes_server_create
 * allocates what aes_serve_run allocates per call (the device key table,
 * per-stream pinned and device staging, streams and events) on the current
 * device and copies the key set and parameters; aes_server_run plays a trace
 * on it exactly as aes_serve_run does, but allocates nothing, and the key
 * cache carries over from one run to the next (the rows stay expanded on
 * the device: a later run's requests for those keys hit); the stats count
 * the run's own hits and misses.  Runs on one server must not overlap (it
 * is not thread-safe).  aes_server_destroy waits for the streams and frees
 * everything; NULL is a no-op.
 *   aes_server_create  errors as aes_serve_run's for the keys and
 *                      parameters, AES_ERR_HIP when a set-up call fails;
 *                      *server_out is NULL unless AES_OK
 *   aes_server_run     errors as aes_serve_run's for the trace, pool and
 *                      output area (key ids checked against the server's
 *                      key set), AES_ERR_NULL for a NULL server
 */
typedef struct aes_server aes_server_t;
aes_status_t aes_server_create(const uint8_t *keys32, const uint8_t *key_len, size_t nkeys,
                               const aes_serve_params_t *params, aes_server_t **server_out);
aes_status_t aes_server_run(aes_server_t *server, const aes_serve_request_t *reqs, size_t nreq,
                            const void *pool_dev, size_t pool_bytes, void *out_dev,
                            size_t out_bytes, double *latency_s, uint64_t *out_off,
                            aes_serve_stats_t *stats);
aes_status_t aes_server_destroy(aes_server_t *server);

/* Text for a status code (static storage). */
const char *aes_status_string(aes_status_t status);

/* Library version, and the number of compute units of the current device
 * (0 when no device is usable). */
const char *aes_version(void);
int aes_device_cu_count(void);

#ifdef __cplusplus
}
#endif

#endif /* AESMI_H */
