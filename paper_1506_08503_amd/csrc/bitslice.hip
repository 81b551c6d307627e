// bitslice.hip -- bitsliced CTR / ECB kernels and launchers; the layout and
// round circuits are described in bitslice_dev.hpp.
#include <hip/hip_runtime.h>

#include "bitslice_dev.hpp"
#include "internal.hpp"

namespace aesmi {
namespace {

// ------------------------------------------------------------------- CTR
template <int NR>
__device__ void ctr_body(const uint32_t *__restrict__ rk, const u32x4 *__restrict__ in,
                         u32x4 *__restrict__ out, uint64_t nbytes, uint32_t n0, uint32_t n1,
                         uint32_t n2, uint32_t ctr0)
{
    const uint64_t nfull = nbytes >> 4;
    const uint32_t tail = (uint32_t)(nbytes & 15u);
    const uint64_t nblk = nfull + (tail ? 1u : 0u);
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t w0 = n0 ^ rk[0], w1 = n1 ^ rk[1], w2 = n2 ^ rk[2];
    for (uint64_t batch = wave; batch * 2048u < nblk; batch += waves)
        bs_ctr_batch<NR>(rk, in, out, nfull, tail, w0, w1, w2, ctr0, batch * 2048u);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void ctr_bitslice_kernel(
    const aes_key_schedule_t *__restrict__ ks, const u32x4 *__restrict__ in,
    u32x4 *__restrict__ out, uint64_t nbytes, uint32_t n0, uint32_t n1, uint32_t n2,
    uint32_t ctr0)
{
    switch (ks->nr) {
    case 10: ctr_body<10>(ks->rk_enc, in, out, nbytes, n0, n1, n2, ctr0); break;
    case 12: ctr_body<12>(ks->rk_enc, in, out, nbytes, n0, n1, n2, ctr0); break;
    case 14: ctr_body<14>(ks->rk_enc, in, out, nbytes, n0, n1, n2, ctr0); break;
    default: break;
    }
}

// ------------------------------------------------------------------- ECB
template <int NR, bool DEC>
__device__ void ecb_body(const uint32_t *__restrict__ rk, const u32x4 *__restrict__ in,
                         u32x4 *__restrict__ out, uint64_t nblocks)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint64_t wave = (uint64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t off = DEC ? kAffine : 0u;
    for (uint64_t batch = wave; batch * 2048u < nblocks; batch += waves) {
        const uint64_t base = batch * 2048u + lane;
        uint32_t p[128];
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const uint64_t i = base + 64u * j;
            const u32x4 v = i < nblocks ? __builtin_nontemporal_load(in + i) : u32x4{0, 0, 0, 0};
            p[j] = v.x ^ rk[0] ^ off;
            p[32 + j] = v.y ^ rk[1] ^ off;
            p[64 + j] = v.z ^ rk[2] ^ off;
            p[96 + j] = v.w ^ rk[3] ^ off;
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            transpose32(p + 32 * c);
        if (DEC)
            decrypt_planes<NR>(p, rk);
        else
            encrypt_planes<NR>(p, rk);
#pragma unroll
        for (int c = 0; c < 4; ++c)
            transpose32(p + 32 * c);
#pragma unroll
        for (int j = 0; j < 32; ++j) {
            const uint64_t i = base + 64u * j;
            if (i < nblocks)
                __builtin_nontemporal_store(u32x4{p[j], p[32 + j], p[64 + j], p[96 + j]}, out + i);
        }
    }
}

template <bool DEC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void ecb_bitslice_kernel(
    const aes_key_schedule_t *__restrict__ ks, const u32x4 *__restrict__ in,
    u32x4 *__restrict__ out, uint64_t nblocks)
{
    const uint32_t *rk = DEC ? ks->rk_dec : ks->rk_enc;
    switch (ks->nr) {
    case 10: ecb_body<10, DEC>(rk, in, out, nblocks); break;
    case 12: ecb_body<12, DEC>(rk, in, out, nblocks); break;
    case 14: ecb_body<14, DEC>(rk, in, out, nblocks); break;
    default: break;
    }
}

struct BsShape {
    uint32_t wg, grid;
};

BsShape resolve(const aes_launch_t *launch, uint64_t nblocks)
{
    // 256-thread workgroups; about 200 VGPRs per lane allow two waves per
    // SIMD, i.e. two resident workgroups per CU.  Each wave takes 2048
    // blocks at a time.  By default the grid has one such batch per wave
    // (up to 64 workgroups per CU): short workgroups that the dispatcher
    // hands to whichever CU is free beat long-lived ones that loop (AES-128
    // CTR over 4 GiB: 953 GB/s with two workgroups per CU, 1039 with 64;
    // AES-256 ECB over 1 GiB: 734 and 777 GB/s).
    BsShape sh{256, 0};
    const int cu = device_cu_count() > 0 ? device_cu_count() : 256;
    uint32_t per_cu = 64;
    if (launch) {
        if (launch->wg_size)
            sh.wg = launch->wg_size;
        if (launch->grid_per_cu)
            per_cu = launch->grid_per_cu;
    }
    const uint64_t per_wg = 2048ull * (sh.wg / 64);
    const uint64_t need = (nblocks + per_wg - 1) / per_wg;
    const uint64_t cap = (uint64_t)cu * per_cu;
    sh.grid = (uint32_t)(need < cap ? (need ? need : 1) : cap);
    return sh;
}

}  // namespace

hipError_t bitslice_ecb(bool decrypt, const aes_key_schedule_t *ks, const void *in, void *out,
                        uint64_t nblocks, const aes_launch_t *launch, hipStream_t stream)
{
    BsShape sh = resolve(launch, nblocks);
    if (sh.wg < 64 || sh.wg > 256 || sh.wg % 64)
        return hipErrorInvalidConfiguration;
    const u32x4 *src = static_cast<const u32x4 *>(in);
    u32x4 *dst = static_cast<u32x4 *>(out);
    if (decrypt)
        hipLaunchKernelGGL(ecb_bitslice_kernel<true>, dim3(sh.grid), dim3(sh.wg), 0, stream, ks,
                           src, dst, nblocks);
    else
        hipLaunchKernelGGL(ecb_bitslice_kernel<false>, dim3(sh.grid), dim3(sh.wg), 0, stream, ks,
                           src, dst, nblocks);
    return hipGetLastError();
}

hipError_t bitslice_ctr(const aes_key_schedule_t *ks, const uint32_t nonce_words[3],
                        uint32_t ctr0, const void *in, void *out, uint64_t nbytes,
                        const aes_launch_t *launch, hipStream_t stream)
{
    BsShape sh = resolve(launch, (nbytes + 15) / 16);
    if (sh.wg < 64 || sh.wg > 256 || sh.wg % 64)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(ctr_bitslice_kernel, dim3(sh.grid), dim3(sh.wg), 0, stream, ks,
                       static_cast<const u32x4 *>(in), static_cast<u32x4 *>(out), nbytes,
                       nonce_words[0], nonce_words[1], nonce_words[2], ctr0);
    return hipGetLastError();
}

}  // namespace aesmi
