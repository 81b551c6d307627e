// bitslice_dev.hpp -- constant-time AES: 32 blocks per lane, one bit per word.
//
// Layout.  Lane l of a wave carries the 32 blocks base + 64 j + l (j = 0..31),
// so every global load or store instruction moves 64 consecutive blocks.
// Inside the lane the 32 blocks are transposed into 128 bit-plane words:
//     P[32 c + b], bit j  =  bit b of column word c of block j,
// i.e. plane 8 k + i holds bit i of state byte k = 4 c + r for all 32 blocks.
// Every step of the round then becomes word-wide boolean logic with no
// data-dependent address anywhere:
//   * SubBytes    -- GF(2^8) inversion + affine map (App. A2) as a tower-field
//                    gate circuit (sbox_circuit.inc, generated from the field
//                    arithmetic), applied to the 8 planes of each byte;
//   * ShiftRows   -- which byte's planes feed which circuit (no data moves);
//   * MixColumns  -- the mix matrix circ[2 3 1 1] (App. A1) on planes: with
//                    d_r = a_r + a_{r+1} and s = a_0 + a_1 + a_2 + a_3,
//                    b_r = 2 d_r + s + a_r, where 2 d is a fixed XOR pattern of
//                    planes (multiplication by x modulo 0x11B);
//   * InvMixColumns -- circ[14 11 13 9] (App. A4) = circ[2 3 1 1] circ[5 0 4 0];
//   * AddRoundKey -- the key is the same for all 32 blocks, so each key bit is
//                    an all-zeros or all-ones word: one XOR per plane.
// The circuits leave out the affine constant 0x63; since the mix matrix maps
// (c, c, c, c) to itself, it is folded into the round keys.
//
// Cost: no LDS tables at all; the S-box is 90 VALU ops (145 gates covered by
// three-input v_bitop3_b32 operations) per byte position per round on 32
// blocks, and a whole AES-128 block takes about 650 VALU ops, three times the
// table kernel's, in exchange for running time and memory traffic that do not
// depend on keys or data.
#pragma once

#include <hip/hip_runtime.h>

#include "aesmi.h"
#include "dev_common.hpp"
#include "sbox_circuit.inc"

namespace aesmi {
namespace {


constexpr uint32_t kAffine = 0x63636363u;

// all-ones if bit b of w is set, else zero
__device__ __forceinline__ uint32_t bitmask(uint32_t w, int b)
{
    return (uint32_t)((int32_t)(w << (31 - b)) >> 31);
}

__device__ __forceinline__ uint32_t mux(uint32_t a, uint32_t b, uint32_t m)
{
    // (a & m) | (b & ~m) in one op
    return __builtin_amdgcn_bitop3_b32(a, b, m, 0xE4);
}

// One stage of the 32 x 32 transpose: swap the S-bit blocks between rows
// k and k + S (for every k with bit S clear).
template <int S>
__device__ __forceinline__ void transpose_stage(uint32_t *a)
{
    const uint32_t m = S == 4 ? 0x0F0F0F0Fu : (S == 2 ? 0x33333333u : 0x55555555u);
#pragma unroll
    for (int blk = 0; blk < 32; blk += 2 * S) {
#pragma unroll
        for (int k = blk; k < blk + S; ++k) {
            const uint32_t lo = a[k], hi = a[k + S];
            if (S == 16) {
                a[k] = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
                a[k + S] = __builtin_amdgcn_perm(hi, lo, 0x07060302u);
            } else if (S == 8) {
                a[k] = __builtin_amdgcn_perm(hi, lo, 0x06020400u);
                a[k + S] = __builtin_amdgcn_perm(hi, lo, 0x07030501u);
            } else {
                a[k] = mux(lo, hi << S, m);
                a[k + S] = mux(lo >> S, hi, m);
            }
        }
    }
}

// In-place 32 x 32 bit transpose: afterwards a[b] bit j = old a[j] bit b.
// Halves and bytes are swapped with byte permutes, nibbles and bits with a
// shift and a masked merge each.
__device__ __forceinline__ void transpose32(uint32_t *a)
{
    transpose_stage<16>(a);
    transpose_stage<8>(a);
    transpose_stage<4>(a);
    transpose_stage<2>(a);
    transpose_stage<1>(a);
}

// SubBytes + ShiftRows: byte (r, c) of q = S'(byte (r, c + r) of p).
__device__ __forceinline__ void sub_shift(const uint32_t *p, uint32_t *q)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int r = k & 3, c = k >> 2;
        const int src = 8 * (r + 4 * ((c + r) & 3));
        const int dst = 8 * k;
        AESMI_SBOX_CIRCUIT(p[src], p[src + 1], p[src + 2], p[src + 3], p[src + 4], p[src + 5],
                           p[src + 6], p[src + 7], q[dst], q[dst + 1], q[dst + 2], q[dst + 3],
                           q[dst + 4], q[dst + 5], q[dst + 6], q[dst + 7]);
    }
}

// InvSubBytes + InvShiftRows: byte (r, c) of q = S'^-1(byte (r, c - r) of p).
__device__ __forceinline__ void inv_sub_shift(const uint32_t *p, uint32_t *q)
{
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int r = k & 3, c = k >> 2;
        const int src = 8 * (r + 4 * ((c - r) & 3));
        const int dst = 8 * k;
        AESMI_INV_SBOX_CIRCUIT(p[src], p[src + 1], p[src + 2], p[src + 3], p[src + 4],
                               p[src + 5], p[src + 6], p[src + 7], q[dst], q[dst + 1],
                               q[dst + 2], q[dst + 3], q[dst + 4], q[dst + 5], q[dst + 6],
                               q[dst + 7]);
    }
}

// p = MixColumns(q) + key, key words k[0..3] (one per column).  Every output
// plane is a 4- or 5-term XOR: two three-input XORs.
__device__ __forceinline__ void mix_add(const uint32_t *q, uint32_t *p, const uint32_t *k)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t *a = q + 32 * c;
        uint32_t d[4][8], s[8];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int i = 0; i < 8; ++i)
                d[r][i] = a[8 * r + i] ^ a[8 * ((r + 1) & 3) + i];
#pragma unroll
        for (int i = 0; i < 8; ++i)
            s[i] = d[0][i] ^ d[2][i];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t *e = d[r];
            // x * e modulo 0x11B: plane i takes e[i-1], and e[7] too for i in {0, 1, 3, 4}
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t m = bitmask(k[c], 8 * r + i);
                const uint32_t ai = a[8 * r + i];
                uint32_t v;
                if (i == 0)
                    v = xor3(e[7], s[0], ai) ^ m;
                else if (i == 1 || i == 3 || i == 4)
                    v = xor3(xor3(e[i - 1], e[7], s[i]), ai, m);
                else
                    v = xor3(e[i - 1], s[i], ai) ^ m;
                p[32 * c + 8 * r + i] = v;
            }
        }
    }
}

// q = circ[5 0 4 0] q in place: a_r + 4 (a_r + a_{r+2}); then MixColumns
// gives InvMixColumns.
__device__ __forceinline__ void inv_mix_pre(uint32_t *q)
{
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        uint32_t *a = q + 32 * c;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            uint32_t t[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                t[i] = a[8 * r + i] ^ a[8 * (r + 2) + i];
            // 4 t modulo 0x11B, plane by plane
            const uint32_t f[8] = {t[6], t[6] ^ t[7], t[0] ^ t[7], t[1] ^ t[6],
                                   t[2] ^ t[6] ^ t[7], t[3] ^ t[7], t[4], t[5]};
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                a[8 * r + i] ^= f[i];
                a[8 * (r + 2) + i] ^= f[i];
            }
        }
    }
}

__device__ __forceinline__ void add_key(uint32_t *p, const uint32_t *q, const uint32_t *k)
{
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int b = 0; b < 32; ++b)
            p[32 * c + b] = q[32 * c + b] ^ bitmask(k[c], b);
}

// Rounds 1..NR on planes that already hold the block XOR round key 0.
template <int NR>
__device__ __forceinline__ void encrypt_planes(uint32_t *p, const uint32_t *rk)
{
#pragma unroll 1
    for (int r = 1; r < NR; ++r) {
        uint32_t q[128];
        sub_shift(p, q);
        const uint32_t k[4] = {rk[4 * r] ^ kAffine, rk[4 * r + 1] ^ kAffine,
                               rk[4 * r + 2] ^ kAffine, rk[4 * r + 3] ^ kAffine};
        mix_add(q, p, k);
    }
    uint32_t q[128];
    sub_shift(p, q);
    const uint32_t k[4] = {rk[4 * NR] ^ kAffine, rk[4 * NR + 1] ^ kAffine,
                           rk[4 * NR + 2] ^ kAffine, rk[4 * NR + 3] ^ kAffine};
    add_key(p, q, k);
}

// Equivalent inverse cipher rounds on planes that hold block XOR dk[0] XOR
// 0x63 (the inverse circuit expects its input offset by the affine constant).
template <int NR>
__device__ __forceinline__ void decrypt_planes(uint32_t *p, const uint32_t *dk)
{
#pragma unroll 1
    for (int r = 1; r < NR; ++r) {
        uint32_t q[128];
        inv_sub_shift(p, q);
        inv_mix_pre(q);
        const uint32_t k[4] = {dk[4 * r] ^ kAffine, dk[4 * r + 1] ^ kAffine,
                               dk[4 * r + 2] ^ kAffine, dk[4 * r + 3] ^ kAffine};
        mix_add(q, p, k);
    }
    uint32_t q[128];
    inv_sub_shift(p, q);
    add_key(p, q, dk + 4 * NR);
}

// One batch of CTR: the 2048 blocks first + 64 j + lane (j = 0..31) of a
// message with nfull whole blocks and a tail of `tail` bytes; w0..w2 are the
// nonce words already XORed with round key 0.  Blocks past the end are
// computed but not stored.
template <int NR>
__device__ __forceinline__ void bs_ctr_batch(const uint32_t *__restrict__ rk,
                                             const u32x4 *__restrict__ in,
                                             u32x4 *__restrict__ out, uint64_t nfull,
                                             uint32_t tail, uint32_t w0, uint32_t w1,
                                             uint32_t w2, uint32_t ctr0, uint64_t first)
{
    const uint64_t base = first + (threadIdx.x & 63u);
    uint32_t p[128];
    // columns 0..2: the nonce, the same in every block
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        p[b] = bitmask(w0, b);
        p[32 + b] = bitmask(w1, b);
        p[64 + b] = bitmask(w2, b);
    }
    // column 3: big-endian counter of block base + 64 j
#pragma unroll
    for (int j = 0; j < 32; ++j)
        p[96 + j] = bswap32(ctr0 + (uint32_t)(base + 64u * j)) ^ rk[3];
    transpose32(p + 96);
    encrypt_planes<NR>(p, rk);
#pragma unroll
    for (int c = 0; c < 4; ++c)
        transpose32(p + 32 * c);
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint64_t i = base + 64u * j;
        const u32x4 ks = {p[j], p[32 + j], p[64 + j], p[96 + j]};
        if (i < nfull) {
            __builtin_nontemporal_store(__builtin_nontemporal_load(in + i) ^ ks, out + i);
        } else if (i == nfull && tail) {
            const uint8_t *src = reinterpret_cast<const uint8_t *>(in + i);
            uint8_t *dst = reinterpret_cast<uint8_t *>(out + i);
            for (uint32_t b = 0; b < tail; ++b)
                dst[b] = src[b] ^ (uint8_t)(ks[b >> 2] >> (8 * (b & 3u)));
        }
    }
}

}  // namespace
}  // namespace aesmi
