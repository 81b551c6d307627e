// ttable_dev.hpp -- AES round function as LDS table lookups (gfx950).
//
// One round of the cipher (sec. II: SubBytes, ShiftRows, MixColumns,
// AddRoundKey) maps the four state columns s_0..s_3 (little-endian words,
// byte j = row j) to
//     s'_c = T0[s_c.b0] ^ T1[s_{c+1}.b1] ^ T2[s_{c+2}.b2] ^ T3[s_{c+3}.b3] ^ k_c
// where Tj[x] is column j of the mix matrix circ[2 3 1 1] (App. A1) times S(x):
// the S-box lookup and the GF(2^8) matrix product of the paper folded into one
// 256-entry table per row.  The last round (no MixColumns, App. A1) takes the
// S-box byte out of the same tables.  Decryption is the equivalent inverse
// cipher with circ[14 11 13 9] (App. A4) tables and an inverse S-box table.
//
// LDS layout (bank-conflict free, 32 copies): copy (lane & 31) of entry x of
// table t sits at byte
//     (t >> 1) << 16 | x << 8 | (t & 1) << 7 | (lane & 31) << 2
// so 32 consecutive lanes always touch 32 distinct banks whatever their bytes,
// and a single v_perm_b32 builds the address from the state word and a
// per-lane constant.  Four encryption tables take 128 KiB; decryption adds a
// 32-copy inverse S-box (32 KiB) at 0x20000: 160 KiB, the whole LDS of a CU.
//
// Work split: each lane carries `bpl` independent blocks per iteration
// (instruction-level parallelism for the LDS latency); a wave touches 64
// consecutive 16-byte blocks per load (1 KiB, one global_load_dwordx4 per
// lane); workgroups stride over the buffer (persistent grid, one workgroup per
// CU because of the LDS footprint).
#pragma once

#include <hip/hip_runtime.h>

#include "aes_tables.hpp"
#include "aesmi.h"
#include "dev_common.hpp"

namespace aesmi {
namespace {

__constant__ Tables g_tab = kTables;


constexpr uint32_t kEncLdsBytes = 4u * 256u * 32u * 4u;          // 131072
constexpr uint32_t kSiBase = 0x20000u;
constexpr uint32_t kDecLdsBytes = kEncLdsBytes + 256u * 32u * 4u;  // 163840

__device__ __forceinline__ uint32_t lds_word(const char *lds, uint32_t byte_addr)
{
    return *reinterpret_cast<const uint32_t *>(lds + byte_addr);
}

// Per-lane address constant of table t: bytes 0 and 2 of the LDS address.
__device__ __forceinline__ uint32_t lane_const(uint32_t t, uint32_t lane)
{
    return ((t >> 1) << 16) | ((t & 1u) << 7) | ((lane & 31u) << 2);
}

// Address of entry (byte k of w) in table t: byte k of w goes to address byte
// 1, the lane constant supplies bytes 0 and 2, byte 3 is zero.
template <int K>
__device__ __forceinline__ uint32_t taddr(uint32_t w, uint32_t lc)
{
    return __builtin_amdgcn_perm(w, lc, 0x0c020000u | ((4u + K) << 8));
}

struct Lc {
    uint32_t t[4];
};

__device__ __forceinline__ Lc make_lc(uint32_t lane)
{
    Lc lc;
#pragma unroll
    for (int t = 0; t < 4; ++t)
        lc.t[t] = lane_const(t, lane);
    return lc;
}

#define TL(T, W, K) lds_word(lds, taddr<K>((W), lc.t[T]))

// (a | b) ^ c in one op (truth table 0x56).
__device__ __forceinline__ uint32_t or_xor(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x56);
}

// One output column of a table round: t0 ^ t1 ^ t2 ^ t3 ^ k in two ops.
__device__ __forceinline__ uint32_t col5(uint32_t t0, uint32_t t1, uint32_t t2, uint32_t t3,
                                         uint32_t k)
{
    return xor3(xor3(t0, t1, t2), t3, k);
}

// ---------------------------------------------------------------- tables
// Fill the four encryption tables (rotations of te0) into LDS, with 16-byte
// stores: store i writes chunk i & 7 (four copies) of entry x = (i >> 4) & 255
// of table t = (i >> 12) << 1 | (i >> 3) & 1.  Sixteen consecutive lanes then
// write the 16 distinct 16-byte bank groups of a 256-byte line (chunk and
// table parity are address bits 4-7), so the fill runs without bank
// conflicts; with lanes on consecutive entries (256 bytes apart) every store
// hit the same group, 7,168 conflict cycles per workgroup (measured).  The
// decryption inverse S-box (32 copies of a byte replicated to a word, 128
// bytes per entry) is filled the same way: chunk i & 7 of entry i >> 3.
__device__ void fill_tables(char *lds, bool decrypt)
{
    const uint32_t nthreads = blockDim.x;
    for (uint32_t i = threadIdx.x; i < 8192u; i += nthreads) {
        const uint32_t c = i & 7u, tl = (i >> 3) & 1u, x = (i >> 4) & 255u, th = i >> 12;
        const uint32_t t = th << 1 | tl;
        const uint32_t base = decrypt ? g_tab.td0[x] : g_tab.te0[x];
        const uint32_t v = t ? ((base << (8 * t)) | (base >> (32 - 8 * t))) : base;
        const uint32_t addr = th << 16 | x << 8 | tl << 7 | c << 4;
        *reinterpret_cast<u32x4 *>(lds + addr) = u32x4{v, v, v, v};
    }
    if (decrypt) {
        for (uint32_t i = threadIdx.x; i < 2048u; i += nthreads) {
            const uint32_t c = i & 7u, x = i >> 3;
            const uint32_t v = 0x01010101u * g_tab.inv_sbox[x];
            *reinterpret_cast<u32x4 *>(lds + kSiBase + (x << 7) + (c << 4)) = u32x4{v, v, v, v};
        }
    }
}

// ------------------------------------------------------------ encryption
// One middle round on one block, round key words rk[0..3].
__device__ __forceinline__ void enc_round(uint32_t (&s)[4], const uint32_t *rk,
                                          const char *lds, const Lc &lc)
{
    uint32_t n0 = col5(TL(0, s[0], 0), TL(1, s[1], 1), TL(2, s[2], 2), TL(3, s[3], 3), rk[0]);
    uint32_t n1 = col5(TL(0, s[1], 0), TL(1, s[2], 1), TL(2, s[3], 2), TL(3, s[0], 3), rk[1]);
    uint32_t n2 = col5(TL(0, s[2], 0), TL(1, s[3], 1), TL(2, s[0], 2), TL(3, s[1], 3), rk[2]);
    uint32_t n3 = col5(TL(0, s[3], 0), TL(1, s[0], 1), TL(2, s[1], 2), TL(3, s[2], 3), rk[3]);
    s[0] = n0;
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
}

// Last round: S-box bytes only.  T3 holds S(x) in byte 0, T0 in byte 1, T1 in
// byte 2 and T2 in byte 3.
__device__ __forceinline__ uint32_t enc_last_col(uint32_t a, uint32_t b, uint32_t c,
                                                 uint32_t d, uint32_t k, const char *lds,
                                                 const Lc &lc)
{
    uint32_t lo = __builtin_amdgcn_perm(TL(0, b, 1), TL(3, a, 0), 0x0c0c0500u);
    uint32_t hi = __builtin_amdgcn_perm(TL(2, d, 3), TL(1, c, 2), 0x07020c0cu);
    return or_xor(lo, hi, k);
}

__device__ __forceinline__ void enc_last(uint32_t (&s)[4], const uint32_t *rk,
                                         const char *lds, const Lc &lc)
{
    uint32_t n0 = enc_last_col(s[0], s[1], s[2], s[3], rk[0], lds, lc);
    uint32_t n1 = enc_last_col(s[1], s[2], s[3], s[0], rk[1], lds, lc);
    uint32_t n2 = enc_last_col(s[2], s[3], s[0], s[1], rk[2], lds, lc);
    uint32_t n3 = enc_last_col(s[3], s[0], s[1], s[2], rk[3], lds, lc);
    s[0] = n0;
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
}

template <int NR, int FIRST, int BPL>
__device__ __forceinline__ void enc_rounds(uint32_t (&s)[BPL][4], const uint32_t *rk,
                                           const char *lds, const Lc &lc)
{
#pragma unroll
    for (int r = FIRST; r < NR; ++r) {
#pragma unroll
        for (int b = 0; b < BPL; ++b)
            enc_round(s[b], rk + 4 * r, lds, lc);
    }
#pragma unroll
    for (int b = 0; b < BPL; ++b)
        enc_last(s[b], rk + 4 * NR, lds, lc);
}

// ------------------------------------------------------------ decryption
__device__ __forceinline__ void dec_round(uint32_t (&s)[4], const uint32_t *rk,
                                          const char *lds, const Lc &lc)
{
    uint32_t n0 = col5(TL(0, s[0], 0), TL(1, s[3], 1), TL(2, s[2], 2), TL(3, s[1], 3), rk[0]);
    uint32_t n1 = col5(TL(0, s[1], 0), TL(1, s[0], 1), TL(2, s[3], 2), TL(3, s[2], 3), rk[1]);
    uint32_t n2 = col5(TL(0, s[2], 0), TL(1, s[1], 1), TL(2, s[0], 2), TL(3, s[3], 3), rk[2]);
    uint32_t n3 = col5(TL(0, s[3], 0), TL(1, s[2], 1), TL(2, s[1], 2), TL(3, s[0], 3), rk[3]);
    s[0] = n0;
    s[1] = n1;
    s[2] = n2;
    s[3] = n3;
}

// Inverse S-box word (byte replicated 4x) of byte K of w.
template <int K>
__device__ __forceinline__ uint32_t si_word(uint32_t w, const char *lds, uint32_t lcs)
{
    return lds_word(lds, (((w >> (8 * K)) & 255u) << 7) | lcs);
}

__device__ __forceinline__ uint32_t dec_last_col(uint32_t a, uint32_t b, uint32_t c,
                                                 uint32_t d, uint32_t k, const char *lds,
                                                 uint32_t lcs)
{
    uint32_t lo = __builtin_amdgcn_perm(si_word<1>(b, lds, lcs), si_word<0>(a, lds, lcs),
                                        0x0c0c0400u);
    uint32_t hi = __builtin_amdgcn_perm(si_word<3>(d, lds, lcs), si_word<2>(c, lds, lcs),
                                        0x04000c0cu);
    return or_xor(lo, hi, k);
}

template <int NR, int BPL>
__device__ __forceinline__ void dec_rounds(uint32_t (&s)[BPL][4], const uint32_t *dk,
                                           const char *lds, const Lc &lc, uint32_t lcs)
{
#pragma unroll
    for (int r = 1; r < NR; ++r) {
#pragma unroll
        for (int b = 0; b < BPL; ++b)
            dec_round(s[b], dk + 4 * r, lds, lc);
    }
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        const uint32_t *k = dk + 4 * NR;
        uint32_t n0 = dec_last_col(s[b][0], s[b][3], s[b][2], s[b][1], k[0], lds, lcs);
        uint32_t n1 = dec_last_col(s[b][1], s[b][0], s[b][3], s[b][2], k[1], lds, lcs);
        uint32_t n2 = dec_last_col(s[b][2], s[b][1], s[b][0], s[b][3], k[2], lds, lcs);
        uint32_t n3 = dec_last_col(s[b][3], s[b][2], s[b][1], s[b][0], k[3], lds, lcs);
        s[b][0] = n0;
        s[b][1] = n1;
        s[b][2] = n2;
        s[b][3] = n3;
    }
}

// ------------------------------------------------------------- ECB body
// Blocks [0, nblocks) are split into tiles of wg * BPL blocks; whole tiles go
// round-robin over the workgroups with no bounds checks inside (so the BPL
// blocks of a lane stay interleaved), the remainder one block per lane.
template <int NR, bool DEC, int BPL>
__device__ __forceinline__ void ecb_blocks(const uint32_t *rk, const u32x4 *__restrict__ in,
                                           u32x4 *__restrict__ out, uint64_t first,
                                           uint64_t stride, const char *lds, const Lc &lc,
                                           uint32_t lcs)
{
    uint32_t s[BPL][4];
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        u32x4 v = __builtin_nontemporal_load(in + first + b * stride);
        s[b][0] = v.x ^ rk[0];
        s[b][1] = v.y ^ rk[1];
        s[b][2] = v.z ^ rk[2];
        s[b][3] = v.w ^ rk[3];
    }
    if (DEC)
        dec_rounds<NR, BPL>(s, rk, lds, lc, lcs);
    else
        enc_rounds<NR, 1, BPL>(s, rk, lds, lc);
#pragma unroll
    for (int b = 0; b < BPL; ++b)
        __builtin_nontemporal_store(u32x4{s[b][0], s[b][1], s[b][2], s[b][3]},
                                    out + first + b * stride);
}

// ------------------------------------------------------------- CTR body
// Counter block i: nonce words n0..n2 and the big-endian counter (ctr0 + i)
// as column 3.  Columns 0..2 are the same for every block, so the three
// round-1 lookups each output column takes from them are done once per
// thread (P0..P3 below); per block only the four lookups that read column 3
// remain in round 1.  The result is the same cipher, bit for bit.
template <int NR, int BPL>
__device__ __forceinline__ void ctr_blocks(const uint32_t *rk, const u32x4 *__restrict__ in,
                                           u32x4 *__restrict__ out, uint64_t first,
                                           uint64_t stride, uint32_t ctr0, uint32_t p0,
                                           uint32_t p1, uint32_t p2, uint32_t p3,
                                           const char *lds, const Lc &lc)
{
    uint32_t s[BPL][4];
    u32x4 x[BPL];
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        const uint64_t i = first + b * stride;
        x[b] = __builtin_nontemporal_load(in + i);
        const uint32_t w3 = bswap32(ctr0 + (uint32_t)i) ^ rk[3];
        s[b][0] = p0 ^ TL(3, w3, 3);
        s[b][1] = p1 ^ TL(2, w3, 2);
        s[b][2] = p2 ^ TL(1, w3, 1);
        s[b][3] = p3 ^ TL(0, w3, 0);
    }
    enc_rounds<NR, 2, BPL>(s, rk, lds, lc);
#pragma unroll
    for (int b = 0; b < BPL; ++b)
        __builtin_nontemporal_store(u32x4{x[b].x ^ s[b][0], x[b].y ^ s[b][1],
                                          x[b].z ^ s[b][2], x[b].w ^ s[b][3]},
                                    out + first + b * stride);
}

// The same keystream with no precomputation: every round, round 1 included,
// from the full counter block (u0..u2 are the nonce words XOR round key 0).
template <int NR, int BPL>
__device__ __forceinline__ void ctr_blocks_plain(const uint32_t *rk,
                                                 const u32x4 *__restrict__ in,
                                                 u32x4 *__restrict__ out, uint64_t first,
                                                 uint64_t stride, uint32_t ctr0, uint32_t u0,
                                                 uint32_t u1, uint32_t u2, const char *lds,
                                                 const Lc &lc)
{
    uint32_t s[BPL][4];
    u32x4 x[BPL];
#pragma unroll
    for (int b = 0; b < BPL; ++b) {
        const uint64_t i = first + b * stride;
        x[b] = __builtin_nontemporal_load(in + i);
        // an empty asm makes the nonce words opaque here, so the compiler
        // cannot hoist their round-1 lookups out of the loop (which would be
        // the round-1 precomputation this variant is measured without)
        uint32_t a0 = u0, a1 = u1, a2 = u2;
        asm volatile("" : "+v"(a0), "+v"(a1), "+v"(a2));
        s[b][0] = a0;
        s[b][1] = a1;
        s[b][2] = a2;
        s[b][3] = bswap32(ctr0 + (uint32_t)i) ^ rk[3];
    }
    enc_rounds<NR, 1, BPL>(s, rk, lds, lc);
#pragma unroll
    for (int b = 0; b < BPL; ++b)
        __builtin_nontemporal_store(u32x4{x[b].x ^ s[b][0], x[b].y ^ s[b][1],
                                          x[b].z ^ s[b][2], x[b].w ^ s[b][3]},
                                    out + first + b * stride);
}

// Counter groups.  Write the counter of block i as c = ctr0 + i and let the
// blocks of one wave be the 256 counters sharing c >> 8 (four per lane, lane
// l taking low bytes l, l + 64, l + 128, l + 192).  After the initial key
// addition only column 3 of a counter block depends on c, and round 1 reads
// one byte of it per output column:
//   * output column 0 reads the low counter byte only, so it depends on
//     (lane, slot) and on nothing else;
//   * output columns 1..3 read the upper three counter bytes, which are the
//     same for the whole group.
// Round 2 reads one byte of round-1 column 0 per output column, the other
// three bytes coming from columns 1..3; so round-2 output column c is
//     Q_c(group) ^ R_c(lane, slot).
// R is computed once per thread (16 lookups) and Q once per group (15
// lookups; lane l of a wave computes Q of the wave's (l+1)-th next group, so
// one pass serves 64 groups, and a group reads its four words back with
// v_readlane), and each block starts at round 3: 16 * (Nr - 2) lookups
// instead of 16 * Nr - 12.  Same cipher, bit for bit.

// Q (round-2 group words, round key 2 added) of the group whose counters
// share the upper bytes of cg.
__device__ __forceinline__ void ctr_group_q(uint32_t cg, const uint32_t *rk,
                                            const uint32_t (&pre)[4], const char *lds,
                                            const Lc &lc, uint32_t (&q)[4])
{
    const uint32_t w3 = bswap32(cg) ^ rk[3];
    const uint32_t s1 = pre[1] ^ TL(2, w3, 2);
    const uint32_t s2 = pre[2] ^ TL(1, w3, 1);
    const uint32_t s3 = pre[3] ^ TL(0, w3, 0);
    q[0] = xor3(TL(1, s1, 1), TL(2, s2, 2), TL(3, s3, 3)) ^ rk[8];
    q[1] = xor3(TL(0, s1, 0), TL(1, s2, 1), TL(2, s3, 2)) ^ rk[9];
    q[2] = xor3(TL(0, s2, 0), TL(1, s3, 1), TL(3, s1, 3)) ^ rk[10];
    q[3] = xor3(TL(0, s3, 0), TL(2, s1, 2), TL(3, s2, 3)) ^ rk[11];
}

// One group of 256 counter blocks on one wave, Q given (wave-uniform).
template <int NR>
__device__ __forceinline__ void ctr_group(const uint32_t *rk, const u32x4 *__restrict__ in,
                                          u32x4 *__restrict__ out, uint64_t first,
                                          const uint32_t (&q)[4], const uint32_t (&r2)[4][4],
                                          const char *lds, const Lc &lc)
{
    uint32_t s[4][4];
    u32x4 x[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        x[b] = __builtin_nontemporal_load(in + first + 64 * b);
        s[b][0] = q[0] ^ r2[b][0];
        s[b][1] = q[1] ^ r2[b][1];
        s[b][2] = q[2] ^ r2[b][2];
        s[b][3] = q[3] ^ r2[b][3];
    }
    enc_rounds<NR, 3, 4>(s, rk, lds, lc);
#pragma unroll
    for (int b = 0; b < 4; ++b)
        __builtin_nontemporal_store(u32x4{x[b].x ^ s[b][0], x[b].y ^ s[b][1],
                                          x[b].z ^ s[b][2], x[b].w ^ s[b][3]},
                                    out + first + 64 * b);
}

// n groups on one wave: group k starts at block blk0 + 256 step k with
// counter c0 + 256 step k (c0 a multiple of 256); lane l takes blocks l,
// l + 64, l + 128 and l + 192 of each.
template <int NR>
__device__ __forceinline__ void ctr_groups(const uint32_t *rk, const u32x4 *__restrict__ in,
                                           u32x4 *__restrict__ out, uint64_t blk0, uint32_t c0,
                                           uint64_t n, uint64_t step, const uint32_t (&pre)[4],
                                           const uint32_t (&r2)[4][4], const char *lds,
                                           const Lc &lc, uint32_t lane)
{
    uint32_t qv[4] = {0, 0, 0, 0};
    for (uint64_t k = 0; k < n; ++k) {
        const uint32_t j = (uint32_t)k & 63u;
        if (j == 0)   // lanes past the last group compute values nobody reads
            ctr_group_q(c0 + (uint32_t)(256u * step * (k + lane)), rk, pre, lds, lc, qv);
        const uint32_t qg[4] = {(uint32_t)__builtin_amdgcn_readlane((int)qv[0], (int)j),
                                (uint32_t)__builtin_amdgcn_readlane((int)qv[1], (int)j),
                                (uint32_t)__builtin_amdgcn_readlane((int)qv[2], (int)j),
                                (uint32_t)__builtin_amdgcn_readlane((int)qv[3], (int)j)};
        ctr_group<NR>(rk, in, out, blk0 + 256u * step * k + lane, qg, r2, lds, lc);
    }
}

}  // namespace
}  // namespace aesmi
