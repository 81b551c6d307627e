// gcm.hip -- Galois/Counter Mode (NIST SP 800-38D) on top of the CTR kernels.
//
// GCM = CTR encryption from counter block IV || 2 (96-bit IVs) plus the tag
//     T = E_K(IV || 1) ^ GHASH_H(A || pad || C || pad || len(A) || len(C)),
// with H = E_K(0^128) and GHASH_H(X_1..X_m) = sum_i X_i * H^(m-i+1) in
// GF(2^128) modulo x^128 + x^7 + x^2 + x + 1 (SP 800-38D sec. 6.3, 6.4).
//
// Field elements travel as four little-endian words of the 16 bytes ("raw"):
// the coefficient of x^i is bit 7 - i%8 of byte i/8.  Reversing the bits of
// every byte gives the "natural" form, where word j bit k is the coefficient
// of x^(32j+k); squaring and multiplication by x are done there.
//
// Multiplication by a fixed G uses 8-bit tables (Shoup's method): with M[b] =
// b(x) * G for every byte value b, Y * G = sum_k x^(8k) M[Y_k], evaluated by
// Horner from the top byte.  Multiplying the accumulator by x^8 is a byte
// shift of the raw words plus a 256-entry reduction table R[o] for the byte o
// that leaves the top.  The wide passes take two bytes per step with a second
// table M'[b] = b(x) x^8 G: acc <- acc * x^16 ^ M'[Y_(2q+1)] ^ M[Y_2q], two R
// lookups per step (about 110 VALU ops and 16 + 14 LDS reads per block).
// The tables live in LDS, replicated so that lanes never share a bank, each
// address one v_perm_b32 of a data word with a per-lane constant:
//   M, M'  256 entries x 16 copies x 16 B each (t << 16 | b << 8 | c << 4)
//   R      256 entries x 32 copies x 4 B at 0x20000 (o << 7 | lane << 2)
// 160 KiB per workgroup.  Narrow passes and the final wave use one copy of a
// one-byte-step table.
//
// Parallel GHASH.  Pad the sequence with zeros in front to T * J blocks (a
// leading zero block does not change GHASH).  Virtual lane g in [0, T) takes
// blocks g, g + T, g + 2T, ... and runs Horner with G = H^T:
//     Y_g = sum_j X_(g + jT) * (H^T)^(J-1-j).
// Then GHASH_H(X) = sum_g Y_g * H^(T-g) = GHASH_H(Y_0, ..., Y_(T-1)): one pass
// maps the sequence to a T-long sequence with the same GHASH.  Passes repeat
// (T a power of two, so G is one of the squarings H^(2^e)) until at most 64
// values remain; one wave then combines them with a tree (pairs multiplied by
// H, H^2, ..., H^32) and a last multiplication by H.  Wave loads are 64
// consecutive blocks (1 KiB) in every pass.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "ttable_dev.hpp"

namespace aesmi {
namespace {

constexpr uint32_t kMaxPow = 32;
constexpr uint64_t kMaxT = 1ull << 19;       // virtual lanes of the widest pass
constexpr uint64_t kWideMinT = 1ull << 16;   // passes this wide use the replicated tables
constexpr uint32_t kFinalN = 64;             // the final wave combines <= 64 values

struct GcmHdr {
    u32x4 ej0;            // E_K(J0), raw (zero for a bare GHASH)
    u32x4 unused;
    u32x4 pow[kMaxPow];   // H^(2^e), natural form
};

// ------------------------------------------------------------ field helpers
struct V4 {
    uint32_t w[4];
};

__device__ __forceinline__ uint32_t raw_nat(uint32_t w)
{
    return __builtin_bitreverse32(bswap32(w));   // reverse the bits of every byte
}

__device__ __forceinline__ V4 mul_x(V4 v)
{
    const uint32_t c = v.w[3] >> 31;
    v.w[3] = (v.w[3] << 1) | (v.w[2] >> 31);
    v.w[2] = (v.w[2] << 1) | (v.w[1] >> 31);
    v.w[1] = (v.w[1] << 1) | (v.w[0] >> 31);
    v.w[0] = (v.w[0] << 1) ^ (c ? 0x87u : 0u);
    return v;
}

__device__ __forceinline__ uint64_t spread32(uint32_t x)
{
    uint64_t v = x;
    v = (v | (v << 16)) & 0x0000FFFF0000FFFFull;
    v = (v | (v << 8)) & 0x00FF00FF00FF00FFull;
    v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0Full;
    v = (v | (v << 2)) & 0x3333333333333333ull;
    v = (v | (v << 1)) & 0x5555555555555555ull;
    return v;
}

// v^2: squaring over GF(2) moves coefficient i to 2i; the 256-bit result is
// reduced with x^128 = x^7 + x^2 + x + 1 (twice for the few bits that the
// first fold pushes past x^127).
__device__ V4 square(V4 v)
{
    uint32_t p[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint64_t s = spread32(v.w[i]);
        p[2 * i] = (uint32_t)s;
        p[2 * i + 1] = (uint32_t)(s >> 32);
    }
    const uint32_t *h = p + 4;
    V4 r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t prev = i ? h[i - 1] : 0u;
        const uint32_t s1 = (h[i] << 1) | (prev >> 31);
        const uint32_t s2 = (h[i] << 2) | (prev >> 30);
        const uint32_t s7 = (h[i] << 7) | (prev >> 25);
        r.w[i] = p[i] ^ h[i] ^ s1 ^ s2 ^ s7;
    }
    const uint32_t ov = (h[3] >> 31) ^ (h[3] >> 30) ^ (h[3] >> 25);
    r.w[0] ^= ov ^ (ov << 1) ^ (ov << 2) ^ (ov << 7);
    return r;
}

// M[idx] = idx(x) * G in raw form, from the basis G * x^t (natural form); bit
// 7 - t of the byte idx is the coefficient of x^t.
__device__ __forceinline__ u32x4 table_entry(const V4 (&b)[8], uint32_t idx)
{
    V4 acc = {{0u, 0u, 0u, 0u}};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const uint32_t m = 0u - ((idx >> (7 - t)) & 1u);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            acc.w[i] ^= b[t].w[i] & m;
    }
    return u32x4{raw_nat(acc.w[0]), raw_nat(acc.w[1]), raw_nat(acc.w[2]), raw_nat(acc.w[3])};
}

__device__ __forceinline__ void basis8(const u32x4 &g, V4 (&b)[8])
{
    b[0] = V4{{g.x, g.y, g.z, g.w}};
#pragma unroll
    for (int t = 1; t < 8; ++t)
        b[t] = mul_x(b[t - 1]);
}

// Reduction word for the raw byte o shifted out of the top by acc * x^8: its
// coefficients x^(128+t) fold to o(x) * (x^7 + x^2 + x + 1), bytes 0 and 1.
__device__ __forceinline__ uint32_t reduce_entry(uint32_t o)
{
    const uint32_t on = __builtin_bitreverse32(o) >> 24;
    return raw_nat(on ^ (on << 1) ^ (on << 2) ^ (on << 7));
}

// ------------------------------------------------------------ table layouts
// Replicated, bank-conflict-free layout for wide passes (160 KiB, the whole
// LDS of a CU), two bytes per Horner step.  M0[b] = b(x) G and M1[b] =
// b(x) x^8 G, 16 copies of 16 bytes each (table t, entry b, copy c at
// t << 16 | b << 8 | c << 4): ds_read_b128 serves 16 lanes per pass, and
// lanes 0-15 of every pass read 16 distinct 16-byte bank groups.  R with 32
// copies of one word at 0x20000 | o << 7 | (lane & 31) << 2 (32 lanes per
// pass for ds_read_b32).  M addresses are one v_perm_b32, R addresses a shift
// and an and-or.
struct WideLayout {
    static constexpr uint32_t kLds = 0x28000u;
    uint32_t c0, c1, cr;

    __device__ explicit WideLayout(uint32_t tid)
        : c0((tid & 15u) << 4), c1(0x10000u | ((tid & 15u) << 4)),
          cr(0x20000u | ((tid & 31u) << 2))
    {
    }

    // entry (byte K of w) of M_T
    template <int T, int K>
    __device__ __forceinline__ u32x4 m(const char *lds, uint32_t w) const
    {
        const uint32_t a = __builtin_amdgcn_perm(w, T ? c1 : c0, 0x0c020000u | ((4u + K) << 8));
        return *reinterpret_cast<const u32x4 *>(lds + a);
    }

    // R[byte K of w], K >= 1
    template <int K>
    __device__ __forceinline__ uint32_t r(const char *lds, uint32_t w) const
    {
        const uint32_t a = ((w >> (8 * K - 7)) & 0x7F80u) | cr;
        return *reinterpret_cast<const uint32_t *>(lds + a);
    }

    __device__ static void fill(char *lds, const u32x4 &g)
    {
        V4 b0[8], b1[8];
        basis8(g, b0);
        V4 g8 = mul_x(b0[7]);
        basis8(u32x4{g8.w[0], g8.w[1], g8.w[2], g8.w[3]}, b1);
        for (uint32_t e = threadIdx.x; e < 2u * 256u * 16u; e += blockDim.x) {
            const uint32_t t = e >> 12, idx = (e >> 4) & 255u, c = e & 15u;
            *reinterpret_cast<u32x4 *>(lds + (t << 16) + (idx << 8) + (c << 4)) =
                t ? table_entry(b1, idx) : table_entry(b0, idx);
        }
        for (uint32_t e = threadIdx.x; e < 256u * 32u; e += blockDim.x) {
            const uint32_t o = e >> 5, l = e & 31u;
            *reinterpret_cast<uint32_t *>(lds + 0x20000u + (o << 7) + (l << 2)) = reduce_entry(o);
        }
    }
};

// y <- y * G ^ x with the wide layout: Y * G = sum_q x^(16q) (M1[Y_(2q+1)] ^
// M0[Y_2q]) by Horner over q; acc * x^16 shifts the raw words by two bytes and
// folds the two bytes that leave the top: byte 14 lands on x^128.. (R[o14] in
// bytes 0-1), byte 15 on x^136.. (R[o15] one byte higher).
template <int Q>
__device__ __forceinline__ void wide_pair(const char *lds, const WideLayout &lay,
                                          const uint32_t (&y)[4], u32x4 &m1, u32x4 &m0)
{
    m1 = lay.template m<1, (2 * Q + 1) & 3>(lds, y[(2 * Q + 1) >> 2]);
    m0 = lay.template m<0, (2 * Q) & 3>(lds, y[(2 * Q) >> 2]);
}

__device__ __forceinline__ void gmul_wide(uint32_t (&y)[4], const uint32_t (&x)[4],
                                          const char *lds, const WideLayout &lay)
{
    u32x4 m1, m0;
    wide_pair<7>(lds, lay, y, m1, m0);
    uint32_t a0 = m1.x ^ m0.x, a1 = m1.y ^ m0.y, a2 = m1.z ^ m0.z, a3 = m1.w ^ m0.w;
#define AESMI_WSTEP(Q)                                                              \
    do {                                                                            \
        const uint32_t ra = lay.template r<2>(lds, a3);                             \
        const uint32_t rb = lay.template r<3>(lds, a3) << 8;                        \
        wide_pair<Q>(lds, lay, y, m1, m0);                                          \
        const uint32_t n3 = __builtin_amdgcn_alignbyte(a3, a2, 2);                  \
        const uint32_t n2 = __builtin_amdgcn_alignbyte(a2, a1, 2);                  \
        const uint32_t n1 = __builtin_amdgcn_alignbyte(a1, a0, 2);                  \
        const uint32_t n0 = a0 << 16;                                               \
        a0 = xor3(xor3(n0, ra, rb), m1.x, m0.x);                                    \
        a1 = xor3(n1, m1.y, m0.y);                                                  \
        a2 = xor3(n2, m1.z, m0.z);                                                  \
        a3 = xor3(n3, m1.w, m0.w);                                                  \
    } while (0)
    AESMI_WSTEP(6);
    AESMI_WSTEP(5);
    AESMI_WSTEP(4);
    AESMI_WSTEP(3);
    AESMI_WSTEP(2);
    AESMI_WSTEP(1);
    AESMI_WSTEP(0);
#undef AESMI_WSTEP
    y[0] = a0 ^ x[0];
    y[1] = a1 ^ x[1];
    y[2] = a2 ^ x[2];
    y[3] = a3 ^ x[3];
}

// One copy of each table (4 KiB + 1 KiB) for narrow passes and the final wave.
struct FlatLayout {
    static constexpr uint32_t kLds = 4096u + 1024u;
    uint32_t mbase, rbase;

    __device__ FlatLayout(uint32_t m_base, uint32_t r_base) : mbase(m_base), rbase(r_base) {}

    template <int K>
    __device__ __forceinline__ u32x4 m(const char *lds, uint32_t w) const
    {
        const uint32_t a = mbase + (((w >> (8 * K)) & 255u) << 4);
        return *reinterpret_cast<const u32x4 *>(lds + a);
    }

    __device__ __forceinline__ uint32_t r(const char *lds, uint32_t w3) const
    {
        return *reinterpret_cast<const uint32_t *>(lds + rbase + ((w3 >> 24) << 2));
    }

    __device__ static void fill_m(char *lds, uint32_t base, const u32x4 &g)
    {
        V4 b[8];
        basis8(g, b);
        for (uint32_t idx = threadIdx.x; idx < 256u; idx += blockDim.x)
            *reinterpret_cast<u32x4 *>(lds + base + (idx << 4)) = table_entry(b, idx);
    }

    __device__ static void fill_r(char *lds, uint32_t base)
    {
        for (uint32_t o = threadIdx.x; o < 256u; o += blockDim.x)
            *reinterpret_cast<uint32_t *>(lds + base + (o << 2)) = reduce_entry(o);
    }
};

// y <- y * G ^ x, G the multiplier whose tables the layout addresses.
template <int K, class L>
__device__ __forceinline__ u32x4 m_byte(const char *lds, const L &lay, const uint32_t (&y)[4])
{
    return lay.template m<(K & 3)>(lds, y[K >> 2]);
}

template <class L>
__device__ __forceinline__ void gmul_acc(uint32_t (&y)[4], const uint32_t (&x)[4],
                                         const char *lds, const L &lay)
{
    const u32x4 top = m_byte<15>(lds, lay, y);
    uint32_t a0 = top.x, a1 = top.y, a2 = top.z, a3 = top.w;
#define AESMI_GSTEP(K)                                                              \
    do {                                                                            \
        const uint32_t r = lay.r(lds, a3);                                          \
        const u32x4 mk = m_byte<K>(lds, lay, y);                                    \
        const uint32_t n3 = __builtin_amdgcn_alignbyte(a3, a2, 3);                  \
        const uint32_t n2 = __builtin_amdgcn_alignbyte(a2, a1, 3);                  \
        const uint32_t n1 = __builtin_amdgcn_alignbyte(a1, a0, 3);                  \
        const uint32_t n0 = a0 << 8;                                                \
        if (K) {                                                                    \
            a0 = xor3(n0, r, mk.x);                                                 \
            a1 = n1 ^ mk.y;                                                         \
            a2 = n2 ^ mk.z;                                                         \
            a3 = n3 ^ mk.w;                                                         \
        } else {                                                                    \
            a0 = xor3(n0, r, mk.x) ^ x[0];                                          \
            a1 = xor3(n1, mk.y, x[1]);                                              \
            a2 = xor3(n2, mk.z, x[2]);                                              \
            a3 = xor3(n3, mk.w, x[3]);                                              \
        }                                                                           \
    } while (0)
    AESMI_GSTEP(14);
    AESMI_GSTEP(13);
    AESMI_GSTEP(12);
    AESMI_GSTEP(11);
    AESMI_GSTEP(10);
    AESMI_GSTEP(9);
    AESMI_GSTEP(8);
    AESMI_GSTEP(7);
    AESMI_GSTEP(6);
    AESMI_GSTEP(5);
    AESMI_GSTEP(4);
    AESMI_GSTEP(3);
    AESMI_GSTEP(2);
    AESMI_GSTEP(1);
    AESMI_GSTEP(0);
#undef AESMI_GSTEP
    y[0] = a0;
    y[1] = a1;
    y[2] = a2;
    y[3] = a3;
}

// ------------------------------------------------------------ sources
__device__ __forceinline__ void zero4(uint32_t (&x)[4])
{
    x[0] = x[1] = x[2] = x[3] = 0u;
}

__device__ __forceinline__ void load4(uint32_t (&x)[4], const void *p)
{
    const u32x4 v = *static_cast<const u32x4 *>(p);
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
}

// Bytes [0, len) of a block, len < 16, zero-padded (SP 800-38D pads A and C).
__device__ void load_partial(uint32_t (&x)[4], const uint8_t *p, uint64_t len)
{
    zero4(x);
    for (uint32_t i = 0; i < (uint32_t)len; ++i)
        x[i >> 2] |= (uint32_t)p[i] << (8 * (i & 3));
}

// A plain array of n 16-byte values.
struct ArraySrc {
    static constexpr bool kAllDirect = true;
    const u32x4 *v;

    __device__ __forceinline__ const u32x4 *at(uint64_t u) const
    {
        return v + u;
    }

    __device__ __forceinline__ void load(uint32_t (&x)[4], uint64_t u) const
    {
        load4(x, v + u);
    }

    __device__ __forceinline__ void fetch(uint32_t (&x)[4], int64_t r) const
    {
        if (r < 0)
            zero4(x);
        else
            load(x, (uint64_t)r);
    }
};

// The GHASH input of GCM: A zero-padded, C zero-padded, then the block
// len(A) || len(C) (64-bit big-endian bit counts).
struct GcmSrc {
    const uint8_t *aad;
    const uint8_t *c;
    uint64_t aad_len, c_len;
    uint64_t na_full, na, nc_full, nc;

    __device__ void fetch(uint32_t (&x)[4], int64_t r) const
    {
        if (r < 0)
            zero4(x);
        else
            load(x, (uint64_t)r);
    }

    static constexpr bool kAllDirect = false;

    // Whole ciphertext blocks, u in [na, na + nc_full), load directly.
    __device__ __forceinline__ const u32x4 *at(uint64_t u) const
    {
        return reinterpret_cast<const u32x4 *>(c) + (u - na);
    }

    __device__ void load(uint32_t (&x)[4], uint64_t u) const
    {
        if (u >= na && u - na < nc_full) {
            load4(x, c + 16 * (u - na));
        } else if (u < na_full) {
            load4(x, aad + 16 * u);
        } else if (u < na) {
            load_partial(x, aad + 16 * u, aad_len - 16 * u);
        } else if (u - na < nc) {
            load_partial(x, c + 16 * (u - na), c_len - 16 * (u - na));
        } else {
            const uint64_t ab = aad_len * 8, cb = c_len * 8;
            x[0] = bswap32((uint32_t)(ab >> 32));
            x[1] = bswap32((uint32_t)ab);
            x[2] = bswap32((uint32_t)(cb >> 32));
            x[3] = bswap32((uint32_t)cb);
        }
    }
};

// ------------------------------------------------------------ kernels
// H = E_K(0), E_K(J0) and the squarings H^(2^e), e < npow.  One workgroup.
__global__ __launch_bounds__(1024) void gcm_setup_kernel(const aes_key_schedule_t *__restrict__ ks,
                                                         uint32_t iv0, uint32_t iv1, uint32_t iv2,
                                                         GcmHdr *hdr, uint32_t npow)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    fill_tables(lds, false);
    __syncthreads();
    if (threadIdx.x != 0)
        return;
    const Lc lc = make_lc(0);
    const uint32_t *rk = ks->rk_enc;
    uint32_t s[2][4] = {{rk[0], rk[1], rk[2], rk[3]},
                        {iv0 ^ rk[0], iv1 ^ rk[1], iv2 ^ rk[2], 0x01000000u ^ rk[3]}};
    switch (ks->nr) {
    case 10: enc_rounds<10, 1, 2>(s, rk, lds, lc); break;
    case 12: enc_rounds<12, 1, 2>(s, rk, lds, lc); break;
    case 14: enc_rounds<14, 1, 2>(s, rk, lds, lc); break;
    default: break;
    }
    hdr->ej0 = u32x4{s[1][0], s[1][1], s[1][2], s[1][3]};
    hdr->unused = u32x4{0u, 0u, 0u, 0u};
    V4 p = {{raw_nat(s[0][0]), raw_nat(s[0][1]), raw_nat(s[0][2]), raw_nat(s[0][3])}};
    for (uint32_t e = 0; e < npow; ++e) {
        hdr->pow[e] = u32x4{p.w[0], p.w[1], p.w[2], p.w[3]};
        p = square(p);
    }
}

// Same header for a bare GHASH with a given H (raw words): E(J0) = 0.
__global__ __launch_bounds__(64) void ghash_setup_kernel(uint32_t h0, uint32_t h1, uint32_t h2,
                                                         uint32_t h3, GcmHdr *hdr, uint32_t npow)
{
    if (threadIdx.x != 0)
        return;
    hdr->ej0 = u32x4{0u, 0u, 0u, 0u};
    hdr->unused = u32x4{0u, 0u, 0u, 0u};
    V4 p = {{raw_nat(h0), raw_nat(h1), raw_nat(h2), raw_nat(h3)}};
    for (uint32_t e = 0; e < npow; ++e) {
        hdr->pow[e] = u32x4{p.w[0], p.w[1], p.w[2], p.w[3]};
        p = square(p);
    }
}

// One pass: T = gridDim * blockDim * CH virtual lanes, J blocks each, front
// padding pad < T (so only the first block of a lane can be padding),
// multiplier H^T = pow[e]; writes Y_0..Y_(T-1).
template <class Src, int CH>
__global__ __launch_bounds__(1024) void ghash_pass_wide_kernel(Src src, uint64_t pad, uint64_t T,
                                                               uint64_t J,
                                                               const GcmHdr *__restrict__ hdr,
                                                               uint32_t e, u32x4 *__restrict__ out)
{
    __shared__ __attribute__((aligned(16))) char lds[WideLayout::kLds];
    WideLayout::fill(lds, hdr->pow[e]);
    __syncthreads();
    const WideLayout lay(threadIdx.x);
    const uint64_t nthr = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t y[CH][4];
#pragma unroll
    for (int i = 0; i < CH; ++i)
        src.fetch(y[i], (int64_t)(gid + i * nthr) - (int64_t)pad);
    // Steps [jlo, jhi) read whole ciphertext blocks in every chain of the
    // wave (the wave's 64 lanes take 64 consecutive blocks); they run a loop
    // with plain loads, the few steps outside it the general loader.
    uint64_t jlo = 1, jhi = J;
    if constexpr (!Src::kAllDirect) {
        const int64_t wb = __builtin_amdgcn_readfirstlane((uint32_t)gid);
        const int64_t lo = (int64_t)src.na, hi = (int64_t)(src.na + src.nc_full) - 64;
        int64_t a = 1, b = (int64_t)J;
#pragma unroll
        for (int i = 0; i < CH; ++i) {
            const int64_t u0 = wb + i * (int64_t)nthr - (int64_t)pad;
            const int64_t ja = lo > u0 ? (lo - u0 + (int64_t)T - 1) / (int64_t)T : 0;
            const int64_t jb = hi >= u0 ? (hi - u0) / (int64_t)T + 1 : 0;
            a = ja > a ? ja : a;
            b = jb < b ? jb : b;
        }
        jlo = (uint64_t)a;
        jhi = (uint64_t)(b > a ? b : a);
    }
    for (uint64_t j = 1; j < J;) {
        if (j >= jlo && j < jhi) {
            for (; j < jhi; ++j) {
                uint32_t x[CH][4];
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    load4(x[i], src.at(gid + i * nthr + j * T - pad));
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    gmul_wide(y[i], x[i], lds, lay);
            }
        } else {
            const uint64_t end = j < jlo ? (jlo < J ? jlo : J) : J;
            for (; j < end; ++j) {
                uint32_t x[CH][4];
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    src.load(x[i], gid + i * nthr + j * T - pad);
#pragma unroll
                for (int i = 0; i < CH; ++i)
                    gmul_wide(y[i], x[i], lds, lay);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < CH; ++i)
        out[gid + i * nthr] = u32x4{y[i][0], y[i][1], y[i][2], y[i][3]};
}

template <class Src>
__global__ __launch_bounds__(256) void ghash_pass_flat_kernel(Src src, uint64_t pad, uint64_t T,
                                                              uint64_t J,
                                                              const GcmHdr *__restrict__ hdr,
                                                              uint32_t e, u32x4 *__restrict__ out)
{
    __shared__ __attribute__((aligned(16))) char lds[FlatLayout::kLds];
    FlatLayout::fill_m(lds, 0u, hdr->pow[e]);
    FlatLayout::fill_r(lds, 4096u);
    __syncthreads();
    const FlatLayout lay(0u, 4096u);
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t y[4];
    src.fetch(y, (int64_t)gid - (int64_t)pad);
    for (uint64_t j = 1; j < J; ++j) {
        uint32_t x[4];
        src.load(x, gid + j * T - pad);
        gmul_acc(y, x, lds, lay);
    }
    out[gid] = u32x4{y[0], y[1], y[2], y[3]};
}

// The last n <= 64 values (front-padded to 64): tree over the wave, times H,
// plus E(J0); writes the 16-byte result.
template <class Src>
__global__ __launch_bounds__(64) void ghash_final_kernel(Src src, uint64_t n,
                                                         const GcmHdr *__restrict__ hdr,
                                                         u32x4 *__restrict__ result)
{
    constexpr uint32_t kR = 6u * 4096u;
    __shared__ __attribute__((aligned(16))) char lds[kR + 1024u];
#pragma unroll 1
    for (uint32_t s = 0; s < 6; ++s)
        FlatLayout::fill_m(lds, s * 4096u, hdr->pow[s]);
    FlatLayout::fill_r(lds, kR);
    __syncthreads();
    const uint32_t lane = threadIdx.x;
    uint32_t y[4];
    src.fetch(y, (int64_t)lane - (int64_t)(kFinalN - n));
    // level s: lane i (a multiple of 2^(s+1)) <- Y_i * H^(2^s) ^ Y_(i + 2^s)
#pragma unroll 1
    for (uint32_t s = 0; s < 6; ++s) {
        const int d = 1 << s;
        uint32_t other[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            other[i] = (uint32_t)__shfl_down((int)y[i], d, 64);
        gmul_acc(y, other, lds, FlatLayout(s * 4096u, kR));
    }
    const uint32_t zero[4] = {0u, 0u, 0u, 0u};
    gmul_acc(y, zero, lds, FlatLayout(0u, kR));
    if (lane == 0) {
        const u32x4 k = hdr->ej0;
        *result = u32x4{y[0] ^ k.x, y[1] ^ k.y, y[2] ^ k.z, y[3] ^ k.w};
    }
}

// ------------------------------------------------------------ plan
struct Plan {
    int npass;
    uint64_t n[8], T[8], J[8];
    uint32_t npow;
    size_t off_a, off_b, bytes;
};

uint64_t pow2_floor(uint64_t x)
{
    uint64_t p = 1;
    while (p * 2 <= x)
        p *= 2;
    return p;
}

uint32_t log2u(uint64_t x)
{
    uint32_t e = 0;
    while ((1ull << e) < x)
        ++e;
    return e;
}

constexpr size_t kHdrBytes = 1024;
static_assert(sizeof(GcmHdr) <= kHdrBytes, "header");

Plan make_plan(uint64_t n0)
{
    Plan p{};
    uint64_t n = n0;
    while (n > kFinalN) {
        uint64_t T = pow2_floor(n / 16 > kFinalN ? n / 16 : kFinalN);
        if (T > kMaxT)
            T = kMaxT;
        p.n[p.npass] = n;
        p.T[p.npass] = T;
        p.J[p.npass] = (n + T - 1) / T;
        ++p.npass;
        n = T;
    }
    p.npow = 7;
    if (p.npass && log2u(p.T[0]) + 1 > p.npow)
        p.npow = log2u(p.T[0]) + 1;
    p.off_a = kHdrBytes;
    p.off_b = p.off_a + (p.npass ? (size_t)p.T[0] * 16 : 0);
    p.bytes = p.off_b + (p.npass > 1 ? (size_t)p.T[1] * 16 : 0);
    return p;
}

template <class Src>
hipError_t run_passes(const Plan &p, const Src &src0, char *ws, uint64_t n0, void *result,
                      hipStream_t stream)
{
    const GcmHdr *hdr = reinterpret_cast<const GcmHdr *>(ws);
    u32x4 *buf[2] = {reinterpret_cast<u32x4 *>(ws + p.off_a),
                     reinterpret_cast<u32x4 *>(ws + p.off_b)};
    for (int l = 0; l < p.npass; ++l) {
        const uint64_t T = p.T[l], J = p.J[l], pad = T * J - p.n[l];
        const uint32_t e = log2u(T);
        u32x4 *out = buf[l & 1];
        if (T >= kWideMinT) {
            constexpr int kCh = 2;
            const uint32_t wg = 1024;
            const uint32_t grid = (uint32_t)(T / (kCh * wg));
            if (l == 0)
                hipLaunchKernelGGL((ghash_pass_wide_kernel<Src, kCh>), dim3(grid), dim3(wg), 0,
                                   stream, src0, pad, T, J, hdr, e, out);
            else
                hipLaunchKernelGGL((ghash_pass_wide_kernel<ArraySrc, kCh>), dim3(grid), dim3(wg),
                                   0, stream, ArraySrc{buf[(l - 1) & 1]}, pad, T, J, hdr, e, out);
        } else {
            const uint32_t wg = (uint32_t)(T < 256 ? T : 256);
            const uint32_t grid = (uint32_t)(T / wg);
            if (l == 0)
                hipLaunchKernelGGL((ghash_pass_flat_kernel<Src>), dim3(grid), dim3(wg), 0, stream,
                                   src0, pad, T, J, hdr, e, out);
            else
                hipLaunchKernelGGL((ghash_pass_flat_kernel<ArraySrc>), dim3(grid), dim3(wg), 0,
                                   stream, ArraySrc{buf[(l - 1) & 1]}, pad, T, J, hdr, e, out);
        }
    }
    u32x4 *res = static_cast<u32x4 *>(result);
    if (p.npass == 0)
        hipLaunchKernelGGL((ghash_final_kernel<Src>), dim3(1), dim3(64), 0, stream, src0, n0, hdr,
                           res);
    else
        hipLaunchKernelGGL((ghash_final_kernel<ArraySrc>), dim3(1), dim3(64), 0, stream,
                           ArraySrc{buf[(p.npass - 1) & 1]}, p.T[p.npass - 1], hdr, res);
    return hipGetLastError();
}

uint64_t gcm_blocks(uint64_t aad_len, uint64_t nbytes)
{
    return (aad_len + 15) / 16 + (nbytes + 15) / 16 + 1;
}

}  // namespace

size_t gcm_workspace_bytes(uint64_t aad_len, uint64_t nbytes)
{
    return make_plan(gcm_blocks(aad_len, nbytes)).bytes;
}

size_t ghash_workspace_bytes(uint64_t nblocks)
{
    return make_plan(nblocks).bytes;
}

hipError_t gcm(bool decrypt, const aes_key_schedule_t *ks, const uint32_t iv_words[3],
               const void *aad, uint64_t aad_len, const void *in, void *out, uint64_t nbytes,
               void *tag, void *ws, hipStream_t stream)
{
    const uint64_t n0 = gcm_blocks(aad_len, nbytes);
    const Plan p = make_plan(n0);
    GcmHdr *hdr = static_cast<GcmHdr *>(ws);
    hipLaunchKernelGGL(gcm_setup_kernel, dim3(1), dim3(1024), 0, stream, ks, iv_words[0],
                       iv_words[1], iv_words[2], hdr, p.npow);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
        return err;
    if (!decrypt && nbytes) {
        err = ttable_ctr(ks, iv_words, 2u, in, out, nbytes, nullptr, stream);
        if (err != hipSuccess)
            return err;
    }
    GcmSrc src;
    src.aad = static_cast<const uint8_t *>(aad);
    src.c = static_cast<const uint8_t *>(decrypt ? in : out);
    src.aad_len = aad_len;
    src.c_len = nbytes;
    src.na_full = aad_len / 16;
    src.na = (aad_len + 15) / 16;
    src.nc_full = nbytes / 16;
    src.nc = (nbytes + 15) / 16;
    err = run_passes(p, src, static_cast<char *>(ws), n0, tag, stream);
    if (err != hipSuccess || !decrypt || !nbytes)
        return err;
    return ttable_ctr(ks, iv_words, 2u, in, out, nbytes, nullptr, stream);
}

hipError_t ghash(const uint32_t h_words[4], const void *x, uint64_t nblocks, void *y, void *ws,
                 hipStream_t stream)
{
    const Plan p = make_plan(nblocks);
    hipLaunchKernelGGL(ghash_setup_kernel, dim3(1), dim3(64), 0, stream, h_words[0], h_words[1],
                       h_words[2], h_words[3], static_cast<GcmHdr *>(ws), p.npow);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess)
        return err;
    return run_passes(p, ArraySrc{static_cast<const u32x4 *>(x)}, static_cast<char *>(ws),
                      nblocks, y, stream);
}

}  // namespace aesmi
