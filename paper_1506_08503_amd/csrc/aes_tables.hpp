// aes_tables.hpp -- compile-time AES constants for the host and the device.
//
// Everything is derived here from the field definition of sec. II (bytes are
// polynomials over GF(2), products reduced by x^8 + x^4 + x^3 + x + 1):
//   * exp / log tables of the generator x + 1 (0x03) give products and
//     inverses (inv(0) := 0, as App. A2 / A5 leave it);
//   * the S-box is the affine map of App. A2 applied to the inverse, written
//     with byte rotations: s = v ^ rotl(v,1) ^ rotl(v,2) ^ rotl(v,3) ^ rotl(v,4) ^ 0x63;
//   * the inverse S-box is the inverse permutation;
//   * te0[x] packs the MixColumns column (2, 1, 1, 3) * S(x) (App. A1 mix row
//     [2 3 1 1]) as a little-endian word, byte j = state row j; the other three
//     round tables are its byte rotations;
//   * td0[x] packs (14, 9, 13, 11) * S^-1(x) (App. A4 mix row [14 11 13 9]).
#pragma once

#include <stdint.h>

namespace aesmi {

struct Tables {
    uint8_t sbox[256];
    uint8_t inv_sbox[256];
    uint8_t exp3[510];
    uint8_t log3[256];
    uint32_t te0[256];
    uint32_t td0[256];
};

constexpr uint8_t rotl8(uint8_t v, int n)
{
    return static_cast<uint8_t>((v << n) | (v >> (8 - n)));
}

constexpr Tables make_tables()
{
    Tables t{};
    // Powers of 0x03: p * 3 = p ^ (p * x), with p * x reduced by 0x11B.
    uint8_t p = 1;
    for (int i = 0; i < 255; ++i) {
        t.exp3[i] = p;
        t.exp3[i + 255] = p;
        t.log3[p] = static_cast<uint8_t>(i);
        uint8_t px = static_cast<uint8_t>((p << 1) ^ ((p & 0x80) ? 0x1B : 0x00));
        p = static_cast<uint8_t>(p ^ px);
    }
    auto mul = [&t](uint8_t a, uint8_t b) -> uint8_t {
        if (a == 0 || b == 0)
            return 0;
        return t.exp3[t.log3[a] + t.log3[b]];
    };
    for (int x = 0; x < 256; ++x) {
        uint8_t inv = x ? t.exp3[255 - t.log3[x]] : 0;
        uint8_t s = static_cast<uint8_t>(inv ^ rotl8(inv, 1) ^ rotl8(inv, 2) ^
                                         rotl8(inv, 3) ^ rotl8(inv, 4) ^ 0x63);
        t.sbox[x] = s;
        t.inv_sbox[s] = static_cast<uint8_t>(x);
    }
    for (int x = 0; x < 256; ++x) {
        uint8_t s = t.sbox[x];
        t.te0[x] = static_cast<uint32_t>(mul(2, s)) | (static_cast<uint32_t>(s) << 8) |
                   (static_cast<uint32_t>(s) << 16) |
                   (static_cast<uint32_t>(mul(3, s)) << 24);
        uint8_t si = t.inv_sbox[x];
        t.td0[x] = static_cast<uint32_t>(mul(14, si)) |
                   (static_cast<uint32_t>(mul(9, si)) << 8) |
                   (static_cast<uint32_t>(mul(13, si)) << 16) |
                   (static_cast<uint32_t>(mul(11, si)) << 24);
    }
    return t;
}

inline constexpr Tables kTables = make_tables();

// GF(2^8) product through the log tables (host-side key work only).
constexpr uint8_t gf_mul(uint8_t a, uint8_t b)
{
    return (a == 0 || b == 0) ? 0 : kTables.exp3[kTables.log3[a] + kTables.log3[b]];
}

}  // namespace aesmi
