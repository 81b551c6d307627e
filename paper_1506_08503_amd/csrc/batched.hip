// batched.hip -- many messages, each with its own key, nonce and counter, in
// one persistent launch over a device segment table.
//
// Sec. II lets every row (message) of the plaintext matrix carry its own IV
// and key schedule (the per-row V and K) and vectorizes all rows at once.
// Here rows have uneven lengths, so the unit of work is a tile: tile_blocks
// consecutive 16-byte blocks of one message.  Two kernels run back to back on
// the caller's stream:
//   1. prepare (one workgroup): validates every segment, counts its tiles,
//      writes the exclusive prefix sums tile_start[0..nsegs] and clears the
//      16 claim counters and the status word in the workspace.  Invalid
//      segments get no tiles and set the status word to AES_ERR_SEGMENT (a
//      key schedule without a valid round count is caught by the CTR kernel,
//      which skips the segment's tiles and sets the same status).
//   2. persistent CTR kernel (a fixed grid of workgroups per CU): wave g of
//      W (numbered workgroups fastest) takes tile g first, then claims
//      tiles W + 16 k + p from one of 16 counters p (its own until that
//      runs dry, then the next one its workgroup has not found empty),
//      finds the tile's segment with a 64-way ballot search over tile_start
//      (in LDS samples of it for the table kernel: two rounds for 10^4
//      segments, then one round of global loads), loads that segment's key
//      schedule and nonce, and runs the T-table or the bitsliced round
//      function on the tile.  The LDS tables are filled once per workgroup;
//      they do not depend on the key.
// Neither kernel uses a memset, so the pair can be captured in a HIP graph and
// replayed after the segment table or the data have been rewritten in place.
#include <hip/hip_runtime.h>

#include "bitslice_dev.hpp"
#include "internal.hpp"
#include "ttable_dev.hpp"

#include <mutex>

// Workspace of the allocation-free batched call (aes_ctr_xcrypt_batched_noalloc):
// the header line, the 16 claim-counter lines and tile_start[0..nsegs] for up
// to 65,536 segments, 261 KiB.  Each device holds its own copy from the time
// the library's code object is loaded there until the process ends.  Host
// code never passes this name to a kernel (on the host it is a stand-in, not
// a device address): it takes the device address from hipGetSymbolAddress
// once per device and uses that.
constexpr uint32_t kNoAllocMaxSegs = 65536;
constexpr size_t kScratchBytes =
    (256u * 17u + 4u * ((size_t)kNoAllocMaxSegs + 1u) + 255u) & ~(size_t)255u;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace aesmi {
namespace {

struct WsHeader {
    int32_t status;
    uint32_t ntiles;
    uint32_t tile_blocks;
    uint32_t unused;
};

// Tile counters, each in a line of its own after the header line: atomic adds
// on one address serialize (about 13 ns each, measured), adds on different
// lines proceed side by side.
constexpr uint32_t kClaimParts = 16;
constexpr size_t kCounterStride = 256;
constexpr size_t kWsHeader = kCounterStride * (kClaimParts + 1);

__host__ __device__ __forceinline__ uint32_t *claim_counter(void *ws, uint32_t p)
{
    return reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + kCounterStride * (p + 1));
}

__device__ __forceinline__ uint32_t *tile_start_of(void *ws)
{
    return reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + kWsHeader);
}

// Tiles of one segment, or 0 when it is empty or invalid (then *bad is set).
// The round count of its key schedule is checked by the CTR kernels, which
// skip such a segment's tiles and set the status word.
__device__ __forceinline__ uint32_t segment_tiles(const aes_segment_t &sg, uint32_t nkeys,
                                                  uint32_t tile_blocks, bool *bad)
{
    const uint64_t nblk = (sg.nbytes + 15u) >> 4;
    const bool ok = sg.key_slot < nkeys && sg.reserved == 0 && (sg.in_off & 15u) == 0 &&
                    (sg.out_off & 15u) == 0 && (uint64_t)sg.ctr0 + nblk <= (1ull << 32);
    if (!ok) {
        *bad = true;
        return 0;
    }
    // valid segments have nblk <= 2^32: a 32-bit division unless the rounded
    // count itself needs 33 bits
    if (nblk <= 0xffffffffull - tile_blocks)
        return ((uint32_t)nblk + tile_blocks - 1u) / tile_blocks;
    return (uint32_t)((nblk + tile_blocks - 1) / tile_blocks);
}

constexpr uint32_t kPrepLdsSegs = 12288;   // tile counts kept in LDS up to this many segments
constexpr int kPrepInFlight = 8;           // segments loaded at once per thread

// One workgroup (a multiple of 64 threads).  Pass 1 reads the table
// coalesced (segment s by thread s mod blockDim, several segments in flight)
// and stores each segment's tile count (it does not read the key schedules);
// pass 2 turns contiguous runs of counts into exclusive prefix sums with a
// scan of the per-thread run totals: within each wave by lane shuffles, then
// over the wave totals (one barrier instead of two per doubling step).
__global__ __launch_bounds__(1024) void batched_prepare(const aes_segment_t *__restrict__ segs,
                                                        uint32_t nsegs, uint32_t nkeys, void *ws,
                                                        uint32_t tile_blocks)
{
    __shared__ uint32_t wave_total[16];
    __shared__ uint32_t cnt_lds[kPrepLdsSegs];
    __shared__ int bad_any;
    WsHeader *h = static_cast<WsHeader *>(ws);
    uint32_t *start = tile_start_of(ws);
    uint32_t *cnt = nsegs <= kPrepLdsSegs ? cnt_lds : start;
    const uint32_t nt = blockDim.x, tid = threadIdx.x;
    if (tid == 0)
        bad_any = 0;
    __syncthreads();
    bool bad = false;
    for (uint32_t s0 = tid; s0 < nsegs; s0 += kPrepInFlight * nt) {
        aes_segment_t sg[kPrepInFlight];
#pragma unroll
        for (int k = 0; k < kPrepInFlight; ++k) {
            const uint32_t s = s0 + k * nt;
            if (s < nsegs)
                sg[k] = segs[s];
        }
#pragma unroll
        for (int k = 0; k < kPrepInFlight; ++k) {
            const uint32_t s = s0 + k * nt;
            if (s < nsegs)
                cnt[s] = segment_tiles(sg[k], nkeys, tile_blocks, &bad);
        }
    }
    if (bad)
        bad_any = 1;
    __syncthreads();
    const uint32_t per = (nsegs + nt - 1) / nt;
    const uint32_t lo = min(nsegs, tid * per), hi = min(nsegs, lo + per);
    uint32_t sum = 0;
#pragma unroll 8
    for (uint32_t s = lo; s < hi; ++s)
        sum += cnt[s];
    // inclusive scan of the per-thread sums: inside the wave, then the totals
    // of the waves before this one
    const uint32_t lane = tid & 63u, wave = tid >> 6;
    uint32_t incl = sum;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += v;
    }
    if (lane == 63)
        wave_total[wave] = incl;
    __syncthreads();
    for (uint32_t w = 0; w < wave; ++w)
        incl += wave_total[w];
    uint32_t run = incl - sum;   // exclusive prefix of this run
#pragma unroll 8
    for (uint32_t s = lo; s < hi; ++s) {
        const uint32_t c = cnt[s];
        start[s] = run;
        run += c;
    }
    __syncthreads();
    if (tid < kClaimParts)
        *claim_counter(ws, tid) = 0;
    if (tid == nt - 1) {
        start[nsegs] = incl;
        h->ntiles = incl;
        h->tile_blocks = tile_blocks;
        h->status = bad_any ? (int32_t)AES_ERR_SEGMENT : (int32_t)AES_OK;
    }
}

// Segment holding tile t: the last s in [lo, hi) with start(s) <= t (empty
// segments share their start with the next one), given start(lo) <= t.  Each
// round splits the candidate range into 64 pieces, one per lane, and keeps
// the last piece whose first entry is <= t.
template <class Start>
__device__ __forceinline__ uint32_t ballot_search(const Start &start, uint32_t lo, uint32_t hi,
                                                  uint32_t t, uint32_t lane)
{
    while (hi - lo > 1) {
        const uint32_t step = (hi - lo + 63u) / 64u;
        const uint32_t idx = lo + lane * step;
        const bool ok = idx < hi && start(idx) <= t;
        const uint64_t m = __ballot(ok);
        // lane 0 tests start(lo) <= t, which always holds: m is never 0 on a
        // full wave (the guard keeps lo in range regardless)
        const uint32_t last = m ? 63u - (uint32_t)__clzll((long long)m) : 0u;
        lo += last * step;
        hi = min(lo + step, hi);
    }
    return lo;
}

__device__ __forceinline__ uint32_t find_segment(const uint32_t *__restrict__ start,
                                                 uint32_t nsegs, uint32_t t, uint32_t lane)
{
    return ballot_search([start](uint32_t i) { return start[i]; }, 0, nsegs, t, lane);
}

// The table kernel keeps samples of tile_start in the LDS left beside its
// tables: sample j = tile_start[j * stride], stride = ceil(nsegs / 7168), so
// the search runs in LDS and then, when stride > 1, in one round of global
// loads within the sampled range (10,000 segments: stride 2).  Without the
// samples every tile took three rounds of dependent global loads.  28 KiB
// leave 4 KiB of the CU's 160 KiB free: with 31 KiB (1 KiB free) the serving
// loop's staging kernel (256 bytes of LDS) could no longer run on a CU beside
// the other stream's table kernel, and its average time in the 1,024-row
// closed loop went from 8 to 33 us.
constexpr uint32_t kTileSamples = 7168;

struct TileSamples {
    uint32_t stride, count;
};

__device__ TileSamples load_tile_samples(uint32_t *smp, const uint32_t *__restrict__ start,
                                         uint32_t nsegs)
{
    TileSamples ts;
    ts.stride = nsegs ? (nsegs + kTileSamples - 1) / kTileSamples : 1u;
    ts.count = (nsegs + ts.stride - 1) / ts.stride;
    for (uint32_t j = threadIdx.x; j < ts.count; j += blockDim.x)
        smp[j] = start[j * ts.stride];
    return ts;
}

__device__ __forceinline__ uint32_t find_segment_sampled(const uint32_t *smp,
                                                         const TileSamples &ts,
                                                         const uint32_t *__restrict__ start,
                                                         uint32_t nsegs, uint32_t t,
                                                         uint32_t lane)
{
    const uint32_t j = ballot_search([smp](uint32_t i) { return smp[i]; }, 0, ts.count, t, lane);
    const uint32_t lo = j * ts.stride;
    return ballot_search([start](uint32_t i) { return start[i]; }, lo,
                         min(lo + ts.stride, nsegs), t, lane);
}

// The next tile of a wave after its first (tile g of wave g), or ntiles when
// none is left.  Counter p hands out tiles dyn0 + kClaimParts k + p, one per
// atomic add; a wave starts at counter `part` and moves on to the next one
// when it runs dry, so every tile is taken exactly once and waves that finish
// early take work from the others.  A counter found dry is marked in the
// workgroup's LDS mask `dry`, and the other waves of the workgroup skip it
// without an add: at the end of a launch each workgroup, not each wave, pays
// the dependent adds that find the 16 counters empty (an add is a round trip
// to memory shared by all XCDs).  Measured on the 10^4-message workload
// (1,024-thread workgroups): one counter, 2,048-block tiles 0.480 ms and
// 256-block tiles 2.20 ms (claim bound); static first tiles and 16 counters
// 0.452 and 0.72 ms.  The mask: 64 MiB of lognormal request sizes (2,299
// messages, 5,730 tiles of 1,024 blocks) 92.7 -> 68.8 us, 16,384 messages of
// 4 KiB 125 -> 89 us, 10^4 messages 0.429 ms at 1,024 blocks.  A plain load
// of the counter before each add (to skip adds on exhausted counters) made
// every tile size slower, and claiming chunks of consecutive tiles per add
// was slower at 2048-4096 blocks per tile (waves then stream through
// separate regions).
__device__ __forceinline__ uint32_t claim_tile(void *ws, uint32_t *dry, uint32_t &part,
                                               uint32_t dyn0, uint32_t ntiles, uint32_t lane)
{
    for (uint32_t tried = 0; tried < kClaimParts; ++tried) {
        uint32_t t = ntiles;
        // a counter whose first tile is past the end is never touched
        const uint32_t dm = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(dry, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
        const bool skip = (uint64_t)dyn0 + part >= ntiles || ((dm >> part) & 1u);
        if (!skip) {
            if (lane == 0) {
                const uint64_t t2 = (uint64_t)dyn0 +
                                    (uint64_t)atomicAdd(claim_counter(ws, part), 1u) * kClaimParts +
                                    part;
                if (t2 < ntiles)
                    t = (uint32_t)t2;
                else
                    atomicOr(dry, 1u << part);
            }
            t = __builtin_amdgcn_readfirstlane(t);
            if (t < ntiles)
                return t;
        }
        part = part + 1 == kClaimParts ? 0u : part + 1;
    }
    return ntiles;
}

// Wave index in the grid, workgroups fastest: the first waves of all
// workgroups come before the second ones, so a launch with fewer tiles than
// waves spreads its static first tiles over every CU instead of packing them
// into the first workgroups (100 messages of 32 KiB in 1,024-block tiles on
// 1,024-thread workgroups: 200 tiles, 13 CUs busy and 49.8 us per call when
// numbered the other way, 33.8 us this way).
__device__ __forceinline__ uint32_t grid_wave()
{
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * gridDim.x + blockIdx.x;
}

// First counter a wave claims from: spread over the waves of a workgroup and
// over workgroups.
__device__ __forceinline__ uint32_t first_part()
{
    return (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) + blockIdx.x) % kClaimParts;
}
__device__ __forceinline__ uint32_t grid_waves() { return gridDim.x * (blockDim.x >> 6); }

// A segment whose key schedule has no valid round count: its tiles are
// skipped (the output stays untouched) and the status word says so.  Every
// lane stores the same word: a lane-divergent store here let the compiler
// split the claim loop into per-lane iterations, and the claim and the
// segment search need the whole wave.
__device__ __forceinline__ void report_bad_schedule(WsHeader *h)
{
    h->status = (int32_t)AES_ERR_SEGMENT;
}

struct TileJob {
    const u32x4 *in;
    u32x4 *out;
    const aes_key_schedule_t *ks;
    uint64_t b0, b1, nfull;
    uint32_t tail, ctr0, n0, n1, n2;
};

__device__ __forceinline__ TileJob make_job(const aes_segment_t *__restrict__ segs,
                                            const uint32_t *__restrict__ start, uint32_t s,
                                            uint32_t t, uint32_t tile_blocks,
                                            const aes_key_schedule_t *__restrict__ ks_table,
                                            const uint8_t *in_base, uint8_t *out_base)
{
    const aes_segment_t &sg = segs[s];
    TileJob j;
    const uint64_t nblk = (sg.nbytes + 15u) >> 4;
    j.in = reinterpret_cast<const u32x4 *>(in_base + sg.in_off);
    j.out = reinterpret_cast<u32x4 *>(out_base + sg.out_off);
    j.ks = ks_table + sg.key_slot;
    j.b0 = (uint64_t)(t - start[s]) * tile_blocks;
    j.b1 = min(j.b0 + tile_blocks, nblk);
    j.nfull = sg.nbytes >> 4;
    j.tail = (uint32_t)(sg.nbytes & 15u);
    j.ctr0 = sg.ctr0;
    const uint32_t *nw = reinterpret_cast<const uint32_t *>(sg.nonce);
    j.n0 = nw[0];
    j.n1 = nw[1];
    j.n2 = nw[2];
    return j;
}

// The last blocks [b, b + 64 NB) of a tile, NB per lane in one pass: block i
// (lane (i - b) mod 64, slot (i - b) / 64) is loaded and stored whole when
// i < j.nfull; the message's partial last block, when this tile holds it, is
// enciphered in the same pass and its bytes go out from lanes 0..tail-1; the
// other slots are enciphered and dropped.  One pass with NB independent
// blocks per lane instead of NB dependent passes of one, plus one more for a
// partial block (about 5% on 64 MiB of lognormal request sizes, relative to
// the same bytes in 1 MiB messages).
template <int NR, int NB>
__device__ __forceinline__ void ttable_rest(const TileJob &j, uint64_t b, const uint32_t (&pre)[4],
                                            const char *lds, const Lc &lc, uint32_t lane)
{
    const uint32_t *rk = j.ks->rk_enc;
    uint32_t s[NB][4];
    u32x4 x[NB];
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const uint64_t i = b + lane + 64u * q;
        x[q] = i < j.nfull ? __builtin_nontemporal_load(j.in + i) : u32x4{0, 0, 0, 0};
        const uint32_t w3 = bswap32(j.ctr0 + (uint32_t)i) ^ rk[3];
        s[q][0] = pre[0] ^ TL(3, w3, 3);
        s[q][1] = pre[1] ^ TL(2, w3, 2);
        s[q][2] = pre[2] ^ TL(1, w3, 1);
        s[q][3] = pre[3] ^ TL(0, w3, 0);
    }
    enc_rounds<NR, 2, NB>(s, rk, lds, lc);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const uint64_t i = b + lane + 64u * q;
        if (i < j.nfull)
            __builtin_nontemporal_store(u32x4{x[q].x ^ s[q][0], x[q].y ^ s[q][1],
                                              x[q].z ^ s[q][2], x[q].w ^ s[q][3]},
                                        j.out + i);
    }
    if (j.tail && j.nfull >= b && j.nfull < b + 64u * NB && j.b1 == j.nfull + 1) {
        const uint32_t d = (uint32_t)(j.nfull - b), src_lane = d & 63u, slot = d >> 6;
        uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < NB; ++q)
            if (slot == (uint32_t)q) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    w[c] = (uint32_t)__builtin_amdgcn_readlane((int)s[q][c], (int)src_lane);
            }
        const uint32_t k = lane & 15u;
        const uint32_t wk = k < 8u ? (k < 4u ? w[0] : w[1]) : (k < 12u ? w[2] : w[3]);
        if (lane < j.tail) {
            const uint8_t *src = reinterpret_cast<const uint8_t *>(j.in + j.nfull);
            uint8_t *dst = reinterpret_cast<uint8_t *>(j.out + j.nfull);
            dst[k] = src[k] ^ (uint8_t)(wk >> (8u * (k & 3u)));
        }
    }
}

// Blocks [b0, b1) of one message on one wave with the table kernel.  With
// four blocks per lane: whole 256-counter groups with the round-1/2
// precomputation when the counters are group aligned, four blocks per lane
// otherwise; with two or one: that many blocks per lane and the round-1
// terms of the nonce columns only.  Then the rest, with the partial last
// block, in passes of up to BPL blocks per lane.
template <int NR, int BPL>
__device__ void ttable_tile(const TileJob &j, const char *lds, const Lc &lc, uint32_t lane)
{
    const uint32_t *rk = j.ks->rk_enc;
    const uint32_t u0 = j.n0 ^ rk[0], u1 = j.n1 ^ rk[1], u2 = j.n2 ^ rk[2];
    const uint32_t pre[4] = {xor3(TL(0, u0, 0), TL(1, u1, 1), TL(2, u2, 2)) ^ rk[4],
                             xor3(TL(0, u1, 0), TL(1, u2, 1), TL(3, u0, 3)) ^ rk[5],
                             xor3(TL(0, u2, 0), TL(2, u0, 2), TL(3, u1, 3)) ^ rk[6],
                             xor3(TL(1, u0, 1), TL(2, u1, 2), TL(3, u2, 3)) ^ rk[7]};
    const uint64_t hi = min(j.b1, j.nfull);
    uint64_t b = j.b0;
    if (BPL == 4 && ((j.ctr0 + (uint32_t)b) & 255u) == 0 && b + 256 <= hi) {
        uint32_t r2[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t s0 = pre[0] ^ TL(3, ((lane + 64u * q) << 24) ^ rk[3], 3);
            r2[q][0] = TL(0, s0, 0);
            r2[q][1] = TL(3, s0, 3);
            r2[q][2] = TL(2, s0, 2);
            r2[q][3] = TL(1, s0, 1);
        }
        const uint64_t n = (hi - b) >> 8;
        ctr_groups<NR>(rk, j.in, j.out, b, j.ctr0 + (uint32_t)b, n, 1, pre, r2, lds, lc, lane);
        b += 256u * n;
    }
    if (BPL > 1) {
        for (; b + 64u * BPL <= hi; b += 64u * BPL)
            ctr_blocks<NR, BPL>(rk, j.in, j.out, b + lane, 64, j.ctr0, pre[0], pre[1], pre[2],
                                pre[3], lds, lc);
    }
    // the rest of the tile, the partial last block included (b1 counts it)
    while (b < j.b1) {
        const uint64_t r = j.b1 - b;
        if (BPL >= 4 && r > 192u) {
            ttable_rest<NR, (BPL >= 4 ? 4 : 1)>(j, b, pre, lds, lc, lane);
            b += 256u;
        } else if (BPL >= 4 && r > 128u) {
            ttable_rest<NR, (BPL >= 4 ? 3 : 1)>(j, b, pre, lds, lc, lane);
            b += 192u;
        } else if (BPL >= 2 && r > 64u) {
            ttable_rest<NR, (BPL >= 2 ? 2 : 1)>(j, b, pre, lds, lc, lane);
            b += 128u;
        } else {
            ttable_rest<NR, 1>(j, b, pre, lds, lc, lane);
            b += 64u;
        }
    }
}

template <int BPL>
__global__ __launch_bounds__(1024) void batched_ttable_kernel(
    const aes_segment_t *__restrict__ segs, uint32_t nsegs,
    const aes_key_schedule_t *__restrict__ ks_table, const uint8_t *in_base,
    uint8_t *out_base, void *ws)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    __shared__ uint32_t smp[kTileSamples];
    __shared__ uint32_t dry;
    WsHeader *h = static_cast<WsHeader *>(ws);
    const uint32_t *start = tile_start_of(ws);
    if (threadIdx.x == 0)
        dry = 0;
    fill_tables(lds, false);
    const TileSamples ts = load_tile_samples(smp, start, nsegs);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const Lc lc = make_lc(lane);
    const uint32_t ntiles = h->ntiles, tile_blocks = h->tile_blocks;
    const uint32_t nw = grid_waves();
    uint32_t part = first_part();
    for (uint32_t t = grid_wave(); t < ntiles; t = claim_tile(ws, &dry, part, nw, ntiles, lane)) {
        const uint32_t s = find_segment_sampled(smp, ts, start, nsegs, t, lane);
        const TileJob j = make_job(segs, start, s, t, tile_blocks, ks_table, in_base, out_base);
        switch (j.ks->nr) {
        case 10: ttable_tile<10, BPL>(j, lds, lc, lane); break;
        case 12: ttable_tile<12, BPL>(j, lds, lc, lane); break;
        case 14: ttable_tile<14, BPL>(j, lds, lc, lane); break;
        default: report_bad_schedule(h); break;
        }
    }
}

template <int NR>
__device__ void bitslice_tile(const TileJob &j)
{
    const uint32_t *rk = j.ks->rk_enc;
    const uint32_t w0 = j.n0 ^ rk[0], w1 = j.n1 ^ rk[1], w2 = j.n2 ^ rk[2];
    for (uint64_t c = j.b0; c < j.b1; c += 2048)
        bs_ctr_batch<NR>(rk, j.in, j.out, j.nfull, j.tail, w0, w1, w2, j.ctr0, c);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void batched_bitslice_kernel(
    const aes_segment_t *__restrict__ segs, uint32_t nsegs,
    const aes_key_schedule_t *__restrict__ ks_table, const uint8_t *in_base,
    uint8_t *out_base, void *ws)
{
    __shared__ uint32_t dry;
    const uint32_t lane = threadIdx.x & 63u;
    WsHeader *h = static_cast<WsHeader *>(ws);
    const uint32_t *start = tile_start_of(ws);
    if (threadIdx.x == 0)
        dry = 0;
    __syncthreads();
    const uint32_t ntiles = h->ntiles, tile_blocks = h->tile_blocks;
    const uint32_t nw = grid_waves();
    uint32_t part = first_part();
    for (uint32_t t = grid_wave(); t < ntiles; t = claim_tile(ws, &dry, part, nw, ntiles, lane)) {
        const uint32_t s = find_segment(start, nsegs, t, lane);
        const TileJob j = make_job(segs, start, s, t, tile_blocks, ks_table, in_base, out_base);
        switch (j.ks->nr) {
        case 10: bitslice_tile<10>(j); break;
        case 12: bitslice_tile<12>(j); break;
        case 14: bitslice_tile<14>(j); break;
        default: report_bad_schedule(h); break;
        }
    }
}

}  // namespace

size_t batched_workspace_bytes(uint32_t nsegs)
{
    const size_t bytes = kWsHeader + 4u * ((size_t)nsegs + 1u);
    return (bytes + 255u) & ~(size_t)255u;
}

void batched_prepare_host(const aes_segment_t *segs, uint32_t nsegs, uint32_t tile_blocks,
                          void *ws_host)
{
    WsHeader *h = static_cast<WsHeader *>(ws_host);
    uint32_t *start = reinterpret_cast<uint32_t *>(static_cast<char *>(ws_host) + kWsHeader);
    uint32_t t = 0;
    for (uint32_t s = 0; s < nsegs; ++s) {
        start[s] = t;
        t += (uint32_t)((((segs[s].nbytes + 15u) >> 4) + tile_blocks - 1) / tile_blocks);
    }
    start[nsegs] = t;
    h->status = (int32_t)AES_OK;
    h->ntiles = t;
    h->tile_blocks = tile_blocks;
    for (uint32_t p = 0; p < kClaimParts; ++p)
        *claim_counter(ws_host, p) = 0;
}

hipError_t batched_ctr_prepared(const aes_segment_t *segs, uint32_t nsegs,
                                const aes_key_schedule_t *ks_table, const uint8_t *in_base,
                                uint8_t *out_base, void *ws, hipStream_t stream)
{
    const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
    hipLaunchKernelGGL(batched_ttable_kernel<4>, dim3((uint32_t)cu), dim3(1024), 0, stream, segs,
                       nsegs, ks_table, in_base, out_base, ws);
    return hipGetLastError();
}

hipError_t batched_ctr(const aes_segment_t *segs, uint32_t nsegs,
                       const aes_key_schedule_t *ks_table, uint32_t nkeys,
                       const uint8_t *in_base, uint8_t *out_base,
                       const aes_batch_tune_t *tune, void *ws, hipStream_t stream)
{
    uint32_t layout = tune ? tune->layout : 0u;
    if (layout == AES_LAYOUT_AUTO)
        layout = AES_LAYOUT_TTABLE;
    const bool bs = layout == AES_LAYOUT_BITSLICE;
    uint32_t wg = tune && tune->wg_size ? tune->wg_size : (bs ? 256u : 1024u);
    uint32_t per_cu = tune && tune->grid_per_cu ? tune->grid_per_cu : (bs ? 2u : 1u);
    uint32_t tile = tune && tune->tile_blocks ? tune->tile_blocks
                                              : (bs ? kBatchedBitsliceTileBlocks : kBatchedTileBlocks);
    const uint32_t bpl = tune && tune->blocks_per_lane ? tune->blocks_per_lane : 4u;
    if (bpl != 1 && bpl != 2 && bpl != 4)
        return hipErrorInvalidConfiguration;
    if (wg < 64 || wg % 64 || wg > (bs ? 256u : 1024u))
        return hipErrorInvalidConfiguration;
    if (bs && tile % 2048u)
        return hipErrorInvalidConfiguration;
    if (tile % 64u)
        return hipErrorInvalidConfiguration;
    const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
    hipLaunchKernelGGL(batched_prepare, dim3(1), dim3(1024), 0, stream, segs, nsegs, nkeys, ws,
                       tile);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const uint32_t grid = (uint32_t)cu * per_cu;
    if (bs)
        hipLaunchKernelGGL(batched_bitslice_kernel, dim3(grid), dim3(wg), 0, stream, segs, nsegs,
                           ks_table, in_base, out_base, ws);
    else if (bpl == 4)
        hipLaunchKernelGGL(batched_ttable_kernel<4>, dim3(grid), dim3(wg), 0, stream, segs, nsegs,
                           ks_table, in_base, out_base, ws);
    else if (bpl == 2)
        hipLaunchKernelGGL(batched_ttable_kernel<2>, dim3(grid), dim3(wg), 0, stream, segs, nsegs,
                           ks_table, in_base, out_base, ws);
    else
        hipLaunchKernelGGL(batched_ttable_kernel<1>, dim3(grid), dim3(wg), 0, stream, segs, nsegs,
                           ks_table, in_base, out_base, ws);
    return hipGetLastError();
}

namespace {

// Copies the status word of a finished batched launch to caller memory.
__global__ void batched_status_copy(const void *ws, int32_t *status)
{
    if (threadIdx.x == 0)
        *status = static_cast<const WsHeader *>(ws)->status;
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
hipError_t scratch_address(void **out)
{
    static std::mutex mu;
    static void *addr[64];
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= 64)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

}  // namespace

uint32_t batched_noalloc_max_segs() { return kNoAllocMaxSegs; }

hipError_t batched_ctr_noalloc(const aes_segment_t *segs, uint32_t nsegs,
                               const aes_key_schedule_t *ks_table, uint32_t nkeys,
                               const uint8_t *in_base, uint8_t *out_base,
                               const aes_batch_tune_t *tune, int32_t *status, hipStream_t stream)
{
    if (nsegs > kNoAllocMaxSegs || batched_workspace_bytes(nsegs) > kScratchBytes)
        return hipErrorInvalidValue;
    void *ws = nullptr;
    hipError_t e = scratch_address(&ws);
    if (e != hipSuccess)
        return e;
    // the prepare kernel clears the claim counters and the status word
    e = batched_ctr(segs, nsegs, ks_table, nkeys, in_base, out_base, tune, ws, stream);
    if (e != hipSuccess || !status)
        return e;
    hipLaunchKernelGGL(batched_status_copy, dim3(1), dim3(64), 0, stream, ws, status);
    return hipGetLastError();
}

}  // namespace aesmi
