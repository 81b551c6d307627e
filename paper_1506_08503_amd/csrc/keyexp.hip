// keyexp.hip -- key expansion of many keys at once, one key per lane.
//
// Used when thousands of messages each bring their own key (the per-row key
// tensor K of sec. II): the schedules are built on the device, next to the
// data, instead of being expanded on the host and copied over.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "aes_tables.hpp"
#include "internal.hpp"
#include "keysched.hpp"

namespace aesmi {
namespace {

__constant__ uint8_t g_sbox[256] = {
#define X(i) kTables.sbox[i]
#define X8(i) X(i), X(i + 1), X(i + 2), X(i + 3), X(i + 4), X(i + 5), X(i + 6), X(i + 7)
#define X64(i) X8(i), X8(i + 8), X8(i + 16), X8(i + 24), X8(i + 32), X8(i + 40), X8(i + 48), X8(i + 56)
    X64(0), X64(64), X64(128), X64(192)
#undef X64
#undef X8
#undef X
};

template <uint32_t NK>
__device__ __forceinline__ void expand_one(const uint8_t *__restrict__ keys, uint64_t k,
                                           aes_key_schedule_t *__restrict__ out,
                                           const uint8_t *sbox)
{
    uint8_t key[4 * NK];
#pragma unroll
    for (uint32_t i = 0; i < 4 * NK; ++i)
        key[i] = keys[k * (4 * NK) + i];
    expand_schedule_nk<NK>(key, out + k, sbox);
}

__global__ __launch_bounds__(256) void expand_keys_kernel(const uint8_t *__restrict__ keys,
                                                          uint32_t key_bytes, uint64_t nkeys,
                                                          aes_key_schedule_t *__restrict__ out)
{
    __shared__ uint8_t sbox[256];
    for (uint32_t i = threadIdx.x; i < 256u; i += blockDim.x)
        sbox[i] = g_sbox[i];
    __syncthreads();
    const uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nkeys)
        return;
    if (key_bytes == 16)
        expand_one<4>(keys, k, out, sbox);
    else if (key_bytes == 24)
        expand_one<6>(keys, k, out, sbox);
    else
        expand_one<8>(keys, k, out, sbox);
}

// One key of 4 NK bytes at `key` into the schedule record `out`: round count,
// key size and encryption round keys (the serving table is read by the CTR
// kernel only, so the decryption keys are not computed).
template <uint32_t NK>
__device__ __forceinline__ void expand_enc_at(const uint8_t *__restrict__ key,
                                              aes_key_schedule_t *__restrict__ out,
                                              const uint8_t *sbox)
{
    uint8_t k[4 * NK];
#pragma unroll
    for (uint32_t i = 0; i < 4 * NK; ++i)
        k[i] = key[i];
    expand_schedule_nk<NK, false>(k, out, sbox);
}

// The serving loop's staging step in one launch: copy n16 16-byte words from
// pinned host memory to the device, and expand nfill keys (read from the same
// host staging) into their rows (encryption keys only), so that a batch needs no separate copy and
// no second dependent launch before its CTR kernel.
struct alignas(16) Word16 {
    uint32_t w[4];
};

__global__ __launch_bounds__(256) void stage_expand_kernel(
    const Word16 *__restrict__ src, Word16 *__restrict__ dst, uint32_t n16,
    const uint8_t *__restrict__ keys32, const uint8_t *__restrict__ lens,
    const uint32_t *__restrict__ slots, uint32_t nfill, aes_key_schedule_t *__restrict__ table)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x, nt = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < n16; i += nt)
        dst[i] = src[i];
    if (nfill == 0)
        return;
    __shared__ uint8_t sbox[256];
    for (uint32_t i = threadIdx.x; i < 256u; i += blockDim.x)
        sbox[i] = g_sbox[i];
    __syncthreads();
    for (uint32_t k = tid; k < nfill; k += nt) {
        const uint8_t *key = keys32 + 32u * k;
        aes_key_schedule_t *out = table + slots[k];
        if (lens[k] == 16)
            expand_enc_at<4>(key, out, sbox);
        else if (lens[k] == 24)
            expand_enc_at<6>(key, out, sbox);
        else
            expand_enc_at<8>(key, out, sbox);
    }
}

}  // namespace

hipError_t stage_and_expand(const void *src_host, void *dst_dev, size_t bytes,
                            const uint8_t *keys32, const uint8_t *lens, const uint32_t *slots,
                            uint32_t nfill, aes_key_schedule_t *table, hipStream_t stream)
{
    if (bytes % 16u || bytes / 16u > 0xffffffffull)
        return hipErrorInvalidValue;
    const uint32_t n16 = (uint32_t)(bytes / 16u);
    const uint32_t need = std::max<uint32_t>((n16 + 255u) / 256u, (nfill + 255u) / 256u);
    const uint32_t grid = std::min<uint32_t>(std::max<uint32_t>(need, 1u), 1024u);
    hipLaunchKernelGGL(stage_expand_kernel, dim3(grid), dim3(256), 0, stream,
                       static_cast<const Word16 *>(src_host), static_cast<Word16 *>(dst_dev), n16,
                       keys32, lens, slots, nfill, table);
    return hipGetLastError();
}

hipError_t expand_keys_device(const uint8_t *keys, uint32_t key_bytes, uint64_t nkeys,
                              aes_key_schedule_t *ks, hipStream_t stream)
{
    const uint32_t wg = 256;
    const uint64_t grid = (nkeys + wg - 1) / wg;
    if (grid > 0x7fffffffull)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(expand_keys_kernel, dim3((uint32_t)grid), dim3(wg), 0, stream, keys,
                       key_bytes, nkeys, ks);
    return hipGetLastError();
}

}  // namespace aesmi
