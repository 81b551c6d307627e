// cbc.hip -- CBC over a matrix of messages, the mode the paper implements.
//
// App. A1 / A4 encrypt N messages of M bytes (the rows of an N x M matrix)
// at once: block i of a row is enciphered after adding the previous
// ciphertext block of the same row (the row's IV for block 0), and deciphering
// adds the previous ciphertext block after the inverse cipher.
//   * Encryption is serial along a row and parallel across rows, the
//     chaining value kept in registers: up to 65,536 rows a quad of four
//     lanes per row (one state column each, ShiftRows through DPP quad
//     permutations), above that one lane per row.  With few rows the chain
//     latency decides and the quad roughly halves it; two rows interleaved
//     per lane, for instruction-level parallelism, was slower at every row
//     count.
//   * Decryption has no serial dependence (every ciphertext block is known):
//     one lane per block, like ECB, plus one extra 16-byte load of the
//     previous ciphertext block (or the IV).
// The round functions are the T-table ones of ttable_dev.hpp.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "ttable_dev.hpp"

namespace aesmi {
namespace {

constexpr int kRowsPerLane = 1;
// Up to this many rows the encryption runs four lanes per row.
constexpr uint64_t kQuadRowsMax = 65536;

template <int NR, int MPL>
__device__ void cbc_enc_body(const uint32_t *__restrict__ rk, const u32x4 *__restrict__ in,
                             u32x4 *__restrict__ out, const u32x4 *__restrict__ iv,
                             uint32_t iv_step, uint64_t nmsg, uint64_t nblk, const char *lds,
                             const Lc &lc)
{
    const uint64_t nthreads = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t m0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; m0 < nmsg;
         m0 += nthreads * MPL) {
        uint32_t chain[MPL][4];
        bool valid[MPL];
        uint64_t row[MPL];
#pragma unroll
        for (int j = 0; j < MPL; ++j) {
            row[j] = m0 + j * nthreads;
            valid[j] = row[j] < nmsg;
            const u32x4 v = valid[j] ? iv[row[j] * iv_step] : u32x4{0, 0, 0, 0};
            chain[j][0] = v.x;
            chain[j][1] = v.y;
            chain[j][2] = v.z;
            chain[j][3] = v.w;
        }
        // the next plaintext block is loaded one step ahead, so its memory
        // latency overlaps the rounds of the current block
        u32x4 next[MPL];
#pragma unroll
        for (int j = 0; j < MPL; ++j)
            next[j] = valid[j] ? in[row[j] * nblk] : u32x4{0, 0, 0, 0};
        for (uint64_t b = 0; b < nblk; ++b) {
            uint32_t s[MPL][4];
#pragma unroll
            for (int j = 0; j < MPL; ++j) {
                const u32x4 x = next[j];
                if (b + 1 < nblk)
                    next[j] = valid[j] ? in[row[j] * nblk + b + 1] : u32x4{0, 0, 0, 0};
                s[j][0] = x.x ^ chain[j][0] ^ rk[0];
                s[j][1] = x.y ^ chain[j][1] ^ rk[1];
                s[j][2] = x.z ^ chain[j][2] ^ rk[2];
                s[j][3] = x.w ^ chain[j][3] ^ rk[3];
            }
            enc_rounds<NR, 1, MPL>(s, rk, lds, lc);
#pragma unroll
            for (int j = 0; j < MPL; ++j) {
                chain[j][0] = s[j][0];
                chain[j][1] = s[j][1];
                chain[j][2] = s[j][2];
                chain[j][3] = s[j][3];
                if (valid[j])
                    out[row[j] * nblk + b] = u32x4{s[j][0], s[j][1], s[j][2], s[j][3]};
            }
        }
    }
}

__global__ __launch_bounds__(1024) void cbc_enc_kernel(const aes_key_schedule_t *__restrict__ ks,
                                                       const u32x4 *__restrict__ in,
                                                       u32x4 *__restrict__ out,
                                                       const u32x4 *__restrict__ iv,
                                                       uint32_t iv_step, uint64_t nmsg,
                                                       uint64_t nblk)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    fill_tables(lds, false);
    __syncthreads();
    const Lc lc = make_lc(threadIdx.x & 63u);
    const uint32_t *rk = ks->rk_enc;
    switch (ks->nr) {
    case 10: cbc_enc_body<10, kRowsPerLane>(rk, in, out, iv, iv_step, nmsg, nblk, lds, lc); break;
    case 12: cbc_enc_body<12, kRowsPerLane>(rk, in, out, iv, iv_step, nmsg, nblk, lds, lc); break;
    case 14: cbc_enc_body<14, kRowsPerLane>(rk, in, out, iv, iv_step, nmsg, nblk, lds, lc); break;
    default: break;
    }
}

// Few rows: four lanes per row, lane c of a quad holding state column c, so
// a chained block costs each lane four table reads per round instead of
// sixteen and the chain latency drops.  A round's column c reads byte r of
// column c + r (ShiftRows); the three other columns come from the quad's
// other lanes by DPP quad permutations.  Quads past the last row are idle
// as a whole, so every DPP source lane is active.
constexpr uint32_t kQuadRot1 = 0x39;   // lane c <- lane c + 1 (mod 4)
constexpr uint32_t kQuadRot2 = 0x4E;   // lane c <- lane c + 2
constexpr uint32_t kQuadRot3 = 0x93;   // lane c <- lane c + 3

// Every lane of a quad is active and reads a lane of its own quad, so the
// DPP move has no old value to keep.  update_dpp with an old value of 0 cost
// a v_mov per move, three of the twelve ALU operations of a round on this
// latency-bound chain (128 rows of 1 MiB: 47.2 ms with them, 45.2 without).
template <uint32_t CTRL>
__device__ __forceinline__ uint32_t quad_rot(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

template <int NR>
__device__ void cbc_enc_quad_body(const uint32_t *__restrict__ rk, const uint32_t *__restrict__ in,
                                  uint32_t *__restrict__ out, const uint32_t *__restrict__ iv,
                                  uint32_t iv_step, uint64_t nmsg, uint64_t nblk,
                                  const char *lds, const Lc &lc)
{
    const uint32_t c = threadIdx.x & 3u;
    uint32_t k[NR + 1];
#pragma unroll
    for (int r = 0; r <= NR; ++r)
        k[r] = rk[4 * r + c];
    const uint64_t nquads = ((uint64_t)gridDim.x * blockDim.x) >> 2;
    for (uint64_t row = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2; row < nmsg;
         row += nquads) {
        uint32_t chain = iv[row * iv_step * 4 + c];
        const uint32_t *src = in + row * nblk * 4 + c;
        uint32_t *dst = out + row * nblk * 4 + c;
        uint32_t next = src[0];
        for (uint64_t b = 0; b < nblk; ++b) {
            uint32_t s = next ^ chain ^ k[0];
            if (b + 1 < nblk)
                next = src[4 * (b + 1)];
#pragma unroll
            for (int r = 1; r < NR; ++r) {
                const uint32_t s1 = quad_rot<kQuadRot1>(s), s2 = quad_rot<kQuadRot2>(s),
                               s3 = quad_rot<kQuadRot3>(s);
                s = col5(TL(0, s, 0), TL(1, s1, 1), TL(2, s2, 2), TL(3, s3, 3), k[r]);
            }
            const uint32_t s1 = quad_rot<kQuadRot1>(s), s2 = quad_rot<kQuadRot2>(s),
                           s3 = quad_rot<kQuadRot3>(s);
            s = enc_last_col(s, s1, s2, s3, k[NR], lds, lc);
            chain = s;
            dst[4 * b] = s;
        }
    }
}

__global__ __launch_bounds__(1024) void cbc_enc_quad_kernel(const aes_key_schedule_t *__restrict__ ks,
                                                           const uint32_t *__restrict__ in,
                                                           uint32_t *__restrict__ out,
                                                           const uint32_t *__restrict__ iv,
                                                           uint32_t iv_step, uint64_t nmsg,
                                                           uint64_t nblk)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    fill_tables(lds, false);
    __syncthreads();
    const Lc lc = make_lc(threadIdx.x & 63u);
    const uint32_t *rk = ks->rk_enc;
    switch (ks->nr) {
    case 10: cbc_enc_quad_body<10>(rk, in, out, iv, iv_step, nmsg, nblk, lds, lc); break;
    case 12: cbc_enc_quad_body<12>(rk, in, out, iv, iv_step, nmsg, nblk, lds, lc); break;
    case 14: cbc_enc_quad_body<14>(rk, in, out, iv, iv_step, nmsg, nblk, lds, lc); break;
    default: break;
    }
}

// Block g = row * nblk + b.  Each thread walks g = g0 + k * T; the row and the
// position in the row are advanced incrementally (one division per thread).
template <int NR>
__device__ void cbc_dec_body(const uint32_t *__restrict__ dk, const u32x4 *__restrict__ in,
                             u32x4 *__restrict__ out, const u32x4 *__restrict__ iv,
                             uint32_t iv_step, uint64_t nmsg, uint64_t nblk, const char *lds,
                             const Lc &lc, uint32_t lcs)
{
    const uint64_t total = nmsg * nblk;
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total)
        return;
    uint64_t row = g / nblk, pos = g - row * nblk;
    const uint64_t drow = step / nblk, dpos = step - drow * nblk;
    for (; g < total; g += step) {
        const u32x4 c = in[g];
        const u32x4 prev = pos ? in[g - 1] : iv[row * iv_step];
        uint32_t s[1][4] = {{c.x ^ dk[0], c.y ^ dk[1], c.z ^ dk[2], c.w ^ dk[3]}};
        dec_rounds<NR, 1>(s, dk, lds, lc, lcs);
        out[g] = u32x4{s[0][0] ^ prev.x, s[0][1] ^ prev.y, s[0][2] ^ prev.z, s[0][3] ^ prev.w};
        row += drow;
        pos += dpos;
        if (pos >= nblk) {
            pos -= nblk;
            row += 1;
        }
    }
}

__global__ __launch_bounds__(1024) void cbc_dec_kernel(const aes_key_schedule_t *__restrict__ ks,
                                                       const u32x4 *__restrict__ in,
                                                       u32x4 *__restrict__ out,
                                                       const u32x4 *__restrict__ iv,
                                                       uint32_t iv_step, uint64_t nmsg,
                                                       uint64_t nblk)
{
    __shared__ __attribute__((aligned(16))) char lds[kDecLdsBytes];
    fill_tables(lds, true);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const Lc lc = make_lc(lane);
    const uint32_t lcs = kSiBase | ((lane & 31u) << 2);
    const uint32_t *dk = ks->rk_dec;
    switch (ks->nr) {
    case 10: cbc_dec_body<10>(dk, in, out, iv, iv_step, nmsg, nblk, lds, lc, lcs); break;
    case 12: cbc_dec_body<12>(dk, in, out, iv, iv_step, nmsg, nblk, lds, lc, lcs); break;
    case 14: cbc_dec_body<14>(dk, in, out, iv, iv_step, nmsg, nblk, lds, lc, lcs); break;
    default: break;
    }
}

}  // namespace

hipError_t cbc(bool decrypt, const aes_key_schedule_t *ks, const void *iv, uint32_t iv_step,
               const void *in, void *out, uint64_t nmsg, uint64_t nblk, hipStream_t stream)
{
    const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
    const u32x4 *src = static_cast<const u32x4 *>(in);
    u32x4 *dst = static_cast<u32x4 *>(out);
    const u32x4 *ivp = static_cast<const u32x4 *>(iv);
    if (decrypt) {
        const uint64_t total = nmsg * nblk;
        uint32_t wg = 1024;
        while (wg > 256 && (total + wg - 1) / wg < (uint64_t)cu)
            wg >>= 1;
        const uint64_t need = (total + wg - 1) / wg;
        const uint32_t grid = (uint32_t)(need < (uint64_t)cu ? need : (uint64_t)cu);
        hipLaunchKernelGGL(cbc_dec_kernel, dim3(grid), dim3(wg), 0, stream, ks, src, dst, ivp,
                           iv_step, nmsg, nblk);
    } else if (nmsg <= kQuadRowsMax) {
        // four lanes per row; workgroups of 256 threads (one wave per SIMD),
        // wider when the rows would need more workgroups than CUs: one
        // workgroup fits on a CU next to the tables, and up to kQuadRowsMax
        // rows every row runs at once
        uint32_t wg = 256;
        while (wg < 1024 && 4 * nmsg > (uint64_t)wg * cu)
            wg <<= 1;
        const uint64_t need = (4 * nmsg + wg - 1) / wg;
        const uint32_t grid = (uint32_t)(need < (uint64_t)cu ? need : (uint64_t)cu);
        hipLaunchKernelGGL(cbc_enc_quad_kernel, dim3(grid), dim3(wg), 0, stream, ks,
                           static_cast<const uint32_t *>(in), static_cast<uint32_t *>(out),
                           static_cast<const uint32_t *>(iv), iv_step, nmsg, nblk);
    } else {
        // one lane per row: spread rows over the CUs first
        uint32_t wg = 1024;
        const uint64_t lanes = (nmsg + kRowsPerLane - 1) / kRowsPerLane;
        while (wg > 64 && (lanes + wg - 1) / wg < (uint64_t)cu)
            wg >>= 1;
        const uint64_t need = (lanes + wg - 1) / wg;
        const uint32_t grid = (uint32_t)(need < (uint64_t)cu ? need : (uint64_t)cu);
        hipLaunchKernelGGL(cbc_enc_kernel, dim3(grid), dim3(wg), 0, stream, ks, src, dst, ivp,
                           iv_step, nmsg, nblk);
    }
    return hipGetLastError();
}

}  // namespace aesmi
