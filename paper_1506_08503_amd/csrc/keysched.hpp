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

__host__ __device__ inline uint8_t ks_xtime(uint8_t a)
{
    return static_cast<uint8_t>((a << 1) ^ ((a & 0x80) ? 0x1B : 0x00));
}

__host__ __device__ inline uint8_t ks_mul(uint8_t a, uint8_t b)
{
    uint8_t acc = 0;
    while (b) {
        if (b & 1)
            acc ^= a;
        a = ks_xtime(a);
        b >>= 1;
    }
    return acc;
}

__host__ __device__ inline uint32_t ks_subword(uint32_t w, const uint8_t *sbox)
{
    return static_cast<uint32_t>(sbox[w & 255u]) |
           (static_cast<uint32_t>(sbox[(w >> 8) & 255u]) << 8) |
           (static_cast<uint32_t>(sbox[(w >> 16) & 255u]) << 16) |
           (static_cast<uint32_t>(sbox[w >> 24]) << 24);
}

__host__ __device__ inline uint32_t ks_inv_mix(uint32_t w)
{
    uint8_t a[4] = {static_cast<uint8_t>(w), static_cast<uint8_t>(w >> 8),
                    static_cast<uint8_t>(w >> 16), static_cast<uint8_t>(w >> 24)};
    uint32_t out = 0;
    for (int i = 0; i < 4; ++i) {
        uint8_t v = ks_mul(14, a[i]) ^ ks_mul(11, a[(i + 1) & 3]) ^
                    ks_mul(13, a[(i + 2) & 3]) ^ ks_mul(9, a[(i + 3) & 3]);
        out |= static_cast<uint32_t>(v) << (8 * i);
    }
    return out;
}

// key_bytes must be 16, 24 or 32 (checked by the caller).
__host__ __device__ inline void expand_schedule(const uint8_t *key, uint32_t key_bytes,
                                                aes_key_schedule_t *ks, const uint8_t *sbox)
{
    const uint32_t nk = key_bytes / 4;
    const uint32_t nr = nk + 6;
    const uint32_t nw = 4 * (nr + 1);
    uint32_t w[60];
    for (uint32_t i = 0; i < nk; ++i)
        w[i] = static_cast<uint32_t>(key[4 * i]) | (static_cast<uint32_t>(key[4 * i + 1]) << 8) |
               (static_cast<uint32_t>(key[4 * i + 2]) << 16) |
               (static_cast<uint32_t>(key[4 * i + 3]) << 24);
    uint8_t rcon = 1;
    for (uint32_t i = nk; i < nw; ++i) {
        uint32_t t = w[i - 1];
        if (i % nk == 0) {
            t = ks_subword((t >> 8) | (t << 24), sbox) ^ rcon;
            rcon = ks_xtime(rcon);
        } else if (nk == 8 && i % nk == 4) {
            t = ks_subword(t, sbox);
        }
        w[i] = w[i - nk] ^ t;
    }
    ks->nr = nr;
    ks->key_bytes = key_bytes;
    for (uint32_t i = 0; i < 60; ++i) {
        ks->rk_enc[i] = i < nw ? w[i] : 0u;
        ks->rk_dec[i] = 0u;
    }
    for (uint32_t c = 0; c < 4; ++c) {
        ks->rk_dec[c] = w[4 * nr + c];
        ks->rk_dec[4 * nr + c] = w[c];
    }
    for (uint32_t r = 1; r < nr; ++r)
        for (uint32_t c = 0; c < 4; ++c)
            ks->rk_dec[4 * r + c] = ks_inv_mix(w[4 * (nr - r) + c]);
}

}  // namespace aesmi
