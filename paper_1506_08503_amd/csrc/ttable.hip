// ttable.hip -- T-table ECB and CTR kernels and their launchers (gfx950).
//
// The round function and the LDS table layout live in ttable_dev.hpp.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "ttable_dev.hpp"

namespace aesmi {
namespace {

// Default launch: blocks one wave carries at most, and the workgroups per CU
// that this may ask for (the explicit grid_per_cu limit).
constexpr uint64_t kWaveBlocks = 16384;
constexpr uint64_t kMaxGridPerCu = 64;

template <int NR, bool DEC, int BPL>
__device__ void ecb_body(const aes_key_schedule_t *__restrict__ ks,
                         const u32x4 *__restrict__ in, u32x4 *__restrict__ out,
                         uint64_t nblocks, const char *lds, const Lc &lc, uint32_t lcs)
{
    const uint32_t *rk = DEC ? ks->rk_dec : ks->rk_enc;
    const uint64_t wg = blockDim.x;
    const uint64_t tile = wg * BPL;
    const uint64_t ntiles = nblocks / tile;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        ecb_blocks<NR, DEC, BPL>(rk, in, out, t * tile + threadIdx.x, wg, lds, lc, lcs);
    for (uint64_t i = ntiles * tile + (uint64_t)blockIdx.x * wg + threadIdx.x; i < nblocks;
         i += (uint64_t)gridDim.x * wg)
        ecb_blocks<NR, DEC, 1>(rk, in, out, i, 0, lds, lc, lcs);
}

// Blocks per lane of the default ECB launch (BPL = 0): four for 10 rounds, two
// for 12 and 14 (measured on 1 GiB: with 14 rounds four blocks per lane run
// 7% slower than two, with 10 rounds two run 3% slower than four).
template <int NR, int BPL>
struct EcbBpl {
    static constexpr int value = BPL ? BPL : (NR == 10 ? 4 : 2);
};

template <bool DEC, int BPL>
__global__ __launch_bounds__(1024) void ecb_ttable_kernel(
    const aes_key_schedule_t *__restrict__ ks, const u32x4 *__restrict__ in,
    u32x4 *__restrict__ out, uint64_t nblocks)
{
    __shared__ __attribute__((aligned(16))) char lds[DEC ? kDecLdsBytes : kEncLdsBytes];
    fill_tables(lds, DEC);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const Lc lc = make_lc(lane);
    const uint32_t lcs = kSiBase | ((lane & 31u) << 2);
    switch (ks->nr) {
    case 10: ecb_body<10, DEC, EcbBpl<10, BPL>::value>(ks, in, out, nblocks, lds, lc, lcs); break;
    case 12: ecb_body<12, DEC, EcbBpl<12, BPL>::value>(ks, in, out, nblocks, lds, lc, lcs); break;
    case 14: ecb_body<14, DEC, EcbBpl<14, BPL>::value>(ks, in, out, nblocks, lds, lc, lcs); break;
    default: break;   // not a schedule made by this library: leave out untouched
    }
}

// PRE: the round-1 terms of the nonce columns once per thread (true) or every
// round from the full counter block (false, the measured baseline of the
// precomputation).
template <int NR, int BPL, bool PRE>
__device__ void ctr_body(const aes_key_schedule_t *__restrict__ ks,
                         const u32x4 *__restrict__ in, u32x4 *__restrict__ out,
                         uint64_t nbytes, uint32_t n0, uint32_t n1, uint32_t n2,
                         uint32_t ctr0, const char *lds, const Lc &lc)
{
    const uint32_t *rk = ks->rk_enc;
    const uint32_t u0 = n0 ^ rk[0], u1 = n1 ^ rk[1], u2 = n2 ^ rk[2];
    const uint32_t p0 = xor3(TL(0, u0, 0), TL(1, u1, 1), TL(2, u2, 2)) ^ rk[4];
    const uint32_t p1 = xor3(TL(0, u1, 0), TL(1, u2, 1), TL(3, u0, 3)) ^ rk[5];
    const uint32_t p2 = xor3(TL(0, u2, 0), TL(2, u0, 2), TL(3, u1, 3)) ^ rk[6];
    const uint32_t p3 = xor3(TL(1, u0, 1), TL(2, u1, 2), TL(3, u2, 3)) ^ rk[7];

    const uint64_t nfull = nbytes >> 4;
    const uint64_t wg = blockDim.x;
    const uint64_t tile = wg * BPL;
    const uint64_t ntiles = nfull / tile;
    for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        if (PRE)
            ctr_blocks<NR, BPL>(rk, in, out, t * tile + threadIdx.x, wg, ctr0, p0, p1, p2, p3,
                                lds, lc);
        else
            ctr_blocks_plain<NR, BPL>(rk, in, out, t * tile + threadIdx.x, wg, ctr0, u0, u1,
                                      u2, lds, lc);
    }
    for (uint64_t i = ntiles * tile + (uint64_t)blockIdx.x * wg + threadIdx.x; i < nfull;
         i += (uint64_t)gridDim.x * wg) {
        if (PRE)
            ctr_blocks<NR, 1>(rk, in, out, i, 0, ctr0, p0, p1, p2, p3, lds, lc);
        else
            ctr_blocks_plain<NR, 1>(rk, in, out, i, 0, ctr0, u0, u1, u2, lds, lc);
    }

    // Ragged tail: the first (nbytes % 16) bytes of block nfull.
    const uint32_t tail = (uint32_t)(nbytes & 15u);
    if (tail && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        uint32_t s1[1][4] = {{u0, u1, u2, bswap32(ctr0 + (uint32_t)nfull) ^ rk[3]}};
        enc_rounds<NR, 1, 1>(s1, rk, lds, lc);
        const uint8_t *src = reinterpret_cast<const uint8_t *>(in + nfull);
        uint8_t *dst = reinterpret_cast<uint8_t *>(out + nfull);
        for (uint32_t k = 0; k < tail; ++k)
            dst[k] = src[k] ^ (uint8_t)(s1[0][k >> 2] >> (8 * (k & 3u)));
    }
}

template <int NR>
__device__ void ctr_body_grouped(const aes_key_schedule_t *__restrict__ ks,
                                 const u32x4 *__restrict__ in, u32x4 *__restrict__ out,
                                 uint64_t nbytes, uint32_t n0, uint32_t n1, uint32_t n2,
                                 uint32_t ctr0, const char *lds, const Lc &lc)
{
    const uint32_t *rk = ks->rk_enc;
    const uint32_t u0 = n0 ^ rk[0], u1 = n1 ^ rk[1], u2 = n2 ^ rk[2];
    // round-1 terms that come from the nonce columns (see ctr_body)
    const uint32_t pre[4] = {xor3(TL(0, u0, 0), TL(1, u1, 1), TL(2, u2, 2)) ^ rk[4],
                             xor3(TL(0, u1, 0), TL(1, u2, 1), TL(3, u0, 3)) ^ rk[5],
                             xor3(TL(0, u2, 0), TL(2, u0, 2), TL(3, u1, 3)) ^ rk[6],
                             xor3(TL(1, u0, 1), TL(2, u1, 2), TL(3, u2, 3)) ^ rk[7]};
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t r2[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t lo = lane + 64u * b;                       // low counter byte
        const uint32_t s0 = pre[0] ^ TL(3, (lo << 24) ^ rk[3], 3);  // round-1 column 0
        r2[b][0] = TL(0, s0, 0);
        r2[b][1] = TL(3, s0, 3);
        r2[b][2] = TL(2, s0, 2);
        r2[b][3] = TL(1, s0, 1);
    }

    const uint64_t nfull = nbytes >> 4;
    const uint32_t delta = ctr0 & 255u;            // position of block 0 in its group
    const uint32_t cbase = ctr0 - delta;
    const uint64_t q_first = delta ? 1u : 0u;
    const uint64_t q_end = (delta + nfull) >> 8;
    uint64_t i_lo = nfull, i_hi = nfull;           // blocks covered by whole groups
    if (q_end > q_first) {
        i_lo = 256u * q_first - delta;
        i_hi = 256u * q_end - delta;
        const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
        const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
        const uint64_t q0 = q_first + wave;
        if (q0 < q_end)
            ctr_groups<NR>(rk, in, out, 256u * q0 - delta, cbase + (uint32_t)(256u * q0),
                           (q_end - q0 + waves - 1) / waves, waves, pre, r2, lds, lc, lane);
    }
    // blocks of the partial first and last groups, one per lane
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nedge = i_lo + (nfull - i_hi);
    const uint32_t p0 = pre[0], p1 = pre[1], p2 = pre[2], p3 = pre[3];
    for (uint64_t j = tid; j < nedge; j += nthreads) {
        const uint64_t i = j < i_lo ? j : i_hi + (j - i_lo);
        ctr_blocks<NR, 1>(rk, in, out, i, 0, ctr0, p0, p1, p2, p3, lds, lc);
    }

    const uint32_t tail = (uint32_t)(nbytes & 15u);
    if (tail && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        uint32_t s1[1][4] = {{u0, u1, u2, bswap32(ctr0 + (uint32_t)nfull) ^ rk[3]}};
        enc_rounds<NR, 1, 1>(s1, rk, lds, lc);
        const uint8_t *src = reinterpret_cast<const uint8_t *>(in + nfull);
        uint8_t *dst = reinterpret_cast<uint8_t *>(out + nfull);
        for (uint32_t k = 0; k < tail; ++k)
            dst[k] = src[k] ^ (uint8_t)(s1[0][k >> 2] >> (8 * (k & 3u)));
    }
}

__global__ __launch_bounds__(1024) void ctr_grouped_kernel(
    const aes_key_schedule_t *__restrict__ ks, const u32x4 *__restrict__ in,
    u32x4 *__restrict__ out, uint64_t nbytes, uint32_t n0, uint32_t n1, uint32_t n2,
    uint32_t ctr0)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    fill_tables(lds, false);
    __syncthreads();
    const Lc lc = make_lc(threadIdx.x & 63u);
    switch (ks->nr) {
    case 10: ctr_body_grouped<10>(ks, in, out, nbytes, n0, n1, n2, ctr0, lds, lc); break;
    case 12: ctr_body_grouped<12>(ks, in, out, nbytes, n0, n1, n2, ctr0, lds, lc); break;
    case 14: ctr_body_grouped<14>(ks, in, out, nbytes, n0, n1, n2, ctr0, lds, lc); break;
    default: break;
    }
}

template <int BPL, bool PRE>
__global__ __launch_bounds__(1024) void ctr_ttable_kernel(
    const aes_key_schedule_t *__restrict__ ks, const u32x4 *__restrict__ in,
    u32x4 *__restrict__ out, uint64_t nbytes, uint32_t n0, uint32_t n1, uint32_t n2,
    uint32_t ctr0)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    fill_tables(lds, false);
    __syncthreads();
    const Lc lc = make_lc(threadIdx.x & 63u);
    switch (ks->nr) {
    case 10: ctr_body<10, BPL, PRE>(ks, in, out, nbytes, n0, n1, n2, ctr0, lds, lc); break;
    case 12: ctr_body<12, BPL, PRE>(ks, in, out, nbytes, n0, n1, n2, ctr0, lds, lc); break;
    case 14: ctr_body<14, BPL, PRE>(ks, in, out, nbytes, n0, n1, n2, ctr0, lds, lc); break;
    default: break;
    }
}

// ------------------------------------------------------------- launching
Shape resolve(const aes_launch_t *launch, uint64_t nblocks)
{
    // Default: 1024-thread workgroups (16 waves, the most one CU can hold
    // next to 128 KiB of tables), four blocks per lane, one workgroup per CU
    // -- or more for long inputs, see below.
    Shape sh{1024, 0, 4};
    const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
    uint32_t per_cu = 0;
    if (launch) {
        if (launch->wg_size)
            sh.wg = launch->wg_size;
        if (launch->blocks_per_lane)
            sh.bpl = launch->blocks_per_lane;
        per_cu = launch->grid_per_cu;
    }
    if (!launch || !launch->wg_size) {
        // Small inputs: narrower workgroups so that more CUs get work.
        while (sh.wg > 256 && (nblocks + sh.wg * sh.bpl - 1) / (sh.wg * sh.bpl) < (uint64_t)cu)
            sh.wg >>= 1;
    }
    if (!per_cu) {
        // Long inputs: enough workgroups that each wave carries at most
        // kWaveBlocks blocks.  The CUs do not all run at quite the same
        // speed; with one long-lived workgroup per CU the slowest sets the
        // time, while several shorter ones per CU let the dispatcher hand
        // the later ones to whichever CU is free (AES-128 CTR over 4 GiB:
        // 1659-1679 GB/s with one per CU, 1702-1764 with two to four;
        // ECB over 4 GiB gains 4-6%; at 1 GiB and below one per CU stays
        // the fastest).
        const uint64_t per_round = (uint64_t)cu * (sh.wg / 64u) * kWaveBlocks;
        const uint64_t want = (nblocks + per_round - 1) / per_round;
        per_cu = (uint32_t)(want < 1 ? 1 : want > kMaxGridPerCu ? kMaxGridPerCu : want);
    }
    uint64_t need = (nblocks + (uint64_t)sh.wg * sh.bpl - 1) / ((uint64_t)sh.wg * sh.bpl);
    uint64_t cap = (uint64_t)cu * per_cu;
    sh.grid = (uint32_t)(need < cap ? (need ? need : 1) : cap);
    return sh;
}

bool valid_shape(const Shape &sh)
{
    return sh.wg >= 64 && sh.wg <= 1024 && sh.wg % 64 == 0 &&
           (sh.bpl == 1 || sh.bpl == 2 || sh.bpl == 4) && sh.grid >= 1;
}

}  // namespace

hipError_t ttable_ecb(bool decrypt, const aes_key_schedule_t *ks, const void *in,
                      void *out, uint64_t nblocks, const aes_launch_t *launch,
                      hipStream_t stream)
{
    Shape sh = resolve(launch, nblocks);
    if (!valid_shape(sh))
        return hipErrorInvalidConfiguration;
    const u32x4 *src = static_cast<const u32x4 *>(in);
    u32x4 *dst = static_cast<u32x4 *>(out);
#define LAUNCH_ECB(D, B)                                                                \
    hipLaunchKernelGGL((ecb_ttable_kernel<D, B>), dim3(sh.grid), dim3(sh.wg), 0, stream, \
                       ks, src, dst, nblocks)
    // no explicit blocks_per_lane: the kernel picks it from the round count
    const uint32_t bpl = launch && launch->blocks_per_lane ? sh.bpl : 0u;
    if (decrypt) {
        if (bpl == 1) LAUNCH_ECB(true, 1);
        else if (bpl == 2) LAUNCH_ECB(true, 2);
        else if (bpl == 4) LAUNCH_ECB(true, 4);
        else LAUNCH_ECB(true, 0);
    } else {
        if (bpl == 1) LAUNCH_ECB(false, 1);
        else if (bpl == 2) LAUNCH_ECB(false, 2);
        else if (bpl == 4) LAUNCH_ECB(false, 4);
        else LAUNCH_ECB(false, 0);
    }
#undef LAUNCH_ECB
    return hipGetLastError();
}

hipError_t ttable_ctr(const aes_key_schedule_t *ks, const uint32_t nonce_words[3],
                      uint32_t ctr0, const void *in, void *out, uint64_t nbytes,
                      const aes_launch_t *launch, hipStream_t stream)
{
    Shape sh = resolve(launch, (nbytes + 15) / 16);
    if (!valid_shape(sh))
        return hipErrorInvalidConfiguration;
    const u32x4 *src = static_cast<const u32x4 *>(in);
    u32x4 *dst = static_cast<u32x4 *>(out);
#define LAUNCH_CTR(B, P)                                                                   \
    hipLaunchKernelGGL((ctr_ttable_kernel<B, P>), dim3(sh.grid), dim3(sh.wg), 0, stream, ks, \
                       src, dst, nbytes, nonce_words[0], nonce_words[1], nonce_words[2],     \
                       ctr0)
    const uint32_t pre = launch ? launch->ctr_precompute : 0u;
    if (pre == 2) {                       // no precomputation
        if (sh.bpl == 1) LAUNCH_CTR(1, false);
        else if (sh.bpl == 2) LAUNCH_CTR(2, false);
        else LAUNCH_CTR(4, false);
    } else if (pre == 1 || sh.bpl != 4) { // round-1 nonce terms only
        if (sh.bpl == 1) LAUNCH_CTR(1, true);
        else if (sh.bpl == 2) LAUNCH_CTR(2, true);
        else LAUNCH_CTR(4, true);
    } else {                              // rounds 1 and 2 (256-counter groups)
        hipLaunchKernelGGL(ctr_grouped_kernel, dim3(sh.grid), dim3(sh.wg), 0, stream, ks, src,
                           dst, nbytes, nonce_words[0], nonce_words[1], nonce_words[2], ctr0);
    }
#undef LAUNCH_CTR
    return hipGetLastError();
}

}  // namespace aesmi
