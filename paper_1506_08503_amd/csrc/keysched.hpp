// keysched.hpp -- AES key expansion shared by the host entry point and the
// device batch-expansion kernel.
//
// App. A3 (128-bit keys): each new round key starts from the previous round
// key's last word, rotated by one byte, passed through the S-box and offset by
// the round constant x^(r-1) in its first byte; the remaining words chain by
// addition.  The word recurrence below is the same schedule for Nk = 4 and
// extends it to Nk = 6 and 8 (FIPS-197 sec. 5.2: Nk = 8 adds an S-box pass at
// i mod 8 == 4).  Words are little-endian: byte j of a word is state row j.
//
// The decryption schedule is the one of the equivalent inverse cipher:
// rounds in reverse order, with InvMixColumns (mix row [14 11 13 9], App. A4)
// applied to the inner round keys.
#pragma once

#include <stdint.h>

#include "aesmi.h"

namespace aesmi {

// x * w in GF(2^8) for the four bytes of w at once (reduction by 0x11B).
__host__ __device__ inline uint32_t ks_xtime4(uint32_t w)
{
    return ((w & 0x7f7f7f7fu) << 1) ^ (((w >> 7) & 0x01010101u) * 0x1bu);
}

__host__ __device__ inline uint32_t ks_rotr8(uint32_t w, unsigned s)
{
    return (w >> s) | (w << (32u - s));
}

__host__ __device__ inline uint32_t ks_subword(uint32_t w, const uint8_t *sbox)
{
    return static_cast<uint32_t>(sbox[w & 255u]) |
           (static_cast<uint32_t>(sbox[(w >> 8) & 255u]) << 8) |
           (static_cast<uint32_t>(sbox[(w >> 16) & 255u]) << 16) |
           (static_cast<uint32_t>(sbox[w >> 24]) << 24);
}

// InvMixColumns of one column word: byte i of the result is
// 14 a_i ^ 11 a_(i+1) ^ 13 a_(i+2) ^ 9 a_(i+3) (mix row [14 11 13 9], App. A4);
// the multiples come from the chain a -> 2a -> 4a -> 8a.
__host__ __device__ inline uint32_t ks_inv_mix(uint32_t w)
{
    const uint32_t w2 = ks_xtime4(w), w4 = ks_xtime4(w2), w8 = ks_xtime4(w4);
    const uint32_t w9 = w8 ^ w, w11 = w9 ^ w2, w13 = w9 ^ w4, w14 = w8 ^ w4 ^ w2;
    return w14 ^ ks_rotr8(w11, 8) ^ ks_rotr8(w13, 16) ^ ks_rotr8(w9, 24);
}

// The schedule for Nk = NK key words; every index is a compile-time constant
// so the words stay in registers on the device.  DEC = false leaves rk_dec
// unwritten (for tables that only counter mode reads).
template <uint32_t NK, bool DEC = true>
__host__ __device__ inline void expand_schedule_nk(const uint8_t *key, aes_key_schedule_t *ks,
                                                   const uint8_t *sbox)
{
    constexpr uint32_t nr = NK + 6;
    constexpr uint32_t nw = 4 * (nr + 1);
    uint32_t w[nw];
#pragma unroll
    for (uint32_t i = 0; i < NK; ++i)
        w[i] = static_cast<uint32_t>(key[4 * i]) | (static_cast<uint32_t>(key[4 * i + 1]) << 8) |
               (static_cast<uint32_t>(key[4 * i + 2]) << 16) |
               (static_cast<uint32_t>(key[4 * i + 3]) << 24);
    uint32_t rcon = 1;
#pragma unroll
    for (uint32_t i = NK; i < nw; ++i) {
        uint32_t t = w[i - 1];
        if (i % NK == 0) {
            t = ks_subword((t >> 8) | (t << 24), sbox) ^ rcon;
            rcon = ks_xtime4(rcon) & 0xffu;
        } else if (NK == 8 && i % NK == 4) {
            t = ks_subword(t, sbox);
        }
        w[i] = w[i - NK] ^ t;
    }
    ks->nr = nr;
    ks->key_bytes = 4 * NK;
#pragma unroll
    for (uint32_t i = 0; i < 60; ++i)
        ks->rk_enc[i] = i < nw ? w[i] : 0u;
    if (!DEC)
        return;
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
        ks->rk_dec[c] = w[4 * nr + c];
        ks->rk_dec[4 * nr + c] = w[c];
    }
#pragma unroll
    for (uint32_t r = 1; r < nr; ++r)
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c)
            ks->rk_dec[4 * r + c] = ks_inv_mix(w[4 * (nr - r) + c]);
#pragma unroll
    for (uint32_t i = 4 * (nr + 1); i < 60; ++i)
        ks->rk_dec[i] = 0u;
}

// key_bytes must be 16, 24 or 32 (checked by the caller).
__host__ __device__ inline void expand_schedule(const uint8_t *key, uint32_t key_bytes,
                                                aes_key_schedule_t *ks, const uint8_t *sbox)
{
    if (key_bytes == 16)
        expand_schedule_nk<4>(key, ks, sbox);
    else if (key_bytes == 24)
        expand_schedule_nk<6>(key, ks, sbox);
    else
        expand_schedule_nk<8>(key, ks, sbox);
}

}  // namespace aesmi
