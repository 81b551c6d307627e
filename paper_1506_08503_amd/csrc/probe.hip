// probe.hip -- microbenchmarks that measure the on-chip ceilings the AES
// kernels are held against (built into libaesmi_probe.so, used by the
// benchmark only; not part of the cipher library).
//
//   kind 0, LDS: random 4-byte reads from the 32-copy, lane-private table
//     layout of the T-table kernels (one v_perm_b32 address build per read,
//     16 independent chains per lane, 1,024-thread workgroups, one per CU)
//     -- the rate the table lookups of a round can reach at best;
//   kind 1, rounds: the T-table middle round itself (16 lookups and the
//     three-input XORs per block) on four blocks per lane, with no HBM
//     traffic -- the rate the table kernels' round function can reach;
//   kind 2, VALU: independent chains of three-input XORs (v_bitop3_b32),
//     several workgroups per CU.
// Every probe also reads the shader clock counter (s_memtime) and the
// constant-rate counter (s_memrealtime) at the start and end of wave 0 of
// each workgroup, which gives the clock the chip held during the probe.
#include <hip/hip_runtime.h>

#include <vector>

#include "ttable_dev.hpp"

namespace aesmi {
namespace {

constexpr int kChains = 16;

__device__ __forceinline__ void clock_mark(uint64_t *clk, bool end)
{
    if (threadIdx.x == 0) {
        const uint64_t c = __builtin_amdgcn_s_memtime();
        const uint64_t r = __builtin_amdgcn_s_memrealtime();
        clk[4 * blockIdx.x + (end ? 2 : 0)] = c;
        clk[4 * blockIdx.x + (end ? 3 : 1)] = r;
    }
}

__global__ __launch_bounds__(1024) void lds_probe_kernel(uint32_t iters, uint64_t *clk,
                                                         uint32_t *sink)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    fill_tables(lds, false);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const Lc lc = make_lc(lane);
    uint32_t a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        a[j] = (threadIdx.x * 0x9E3779B9u) ^ (0x01000193u * (uint32_t)(j + 1));
    clock_mark(clk, false);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            a[j] = lds_word(lds, taddr<1>(a[j], lc.t[j & 3]));
    }
    clock_mark(clk, true);
    uint32_t x = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        x ^= a[j];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

__global__ __launch_bounds__(1024) void round_probe_kernel(uint32_t iters, uint64_t *clk,
                                                           uint32_t *sink)
{
    __shared__ __attribute__((aligned(16))) char lds[kEncLdsBytes];
    fill_tables(lds, false);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const Lc lc = make_lc(lane);
    const uint32_t rk[4] = {0x03020100u, 0x07060504u, 0x0b0a0908u, 0x0f0e0d0cu};
    uint32_t s[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            s[b][c] = (threadIdx.x * 0x9E3779B9u) ^ (0x01000193u * (uint32_t)(4 * b + c + 1));
    clock_mark(clk, false);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
            enc_round(s[b], rk, lds, lc);
    }
    clock_mark(clk, true);
    uint32_t x = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        x ^= s[b][0] ^ s[b][1] ^ s[b][2] ^ s[b][3];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

__global__ __launch_bounds__(1024) void valu_probe_kernel(uint32_t iters, uint64_t *clk,
                                                          uint32_t *sink)
{
    uint32_t a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        a[j] = (threadIdx.x * 0x9E3779B9u) ^ (0x01000193u * (uint32_t)(j + 1));
    clock_mark(clk, false);
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kChains; ++j)
            a[j] = xor3(a[j], a[(j + 1) % kChains], a[(j + 5) % kChains] + it);
    }
    clock_mark(clk, true);
    uint32_t x = 0;
#pragma unroll
    for (int j = 0; j < kChains; ++j)
        x ^= a[j];
    sink[blockIdx.x * blockDim.x + threadIdx.x] = x;
}

}  // namespace
}  // namespace aesmi

using namespace aesmi;

extern "C" {

/*
 * aesmi_probe_run -- run one probe (kind 0 LDS, 1 rounds, 2 VALU, see above)
 * with `iters` loop iterations per thread, once untimed and then `reps` times
 * back to back between two events on a private stream.
 *   ms          out: average milliseconds per run
 *   rate        out: operations per second (kind 0: lane reads of 4 bytes;
 *               kind 1: block-rounds; kind 2: lane operations, counting the
 *               add of the loop counter as well as the XOR)
 *   sclk_ghz    out: clock of the shader counter over the timed runs (0 if
 *               the counters could not be read)
 * Returns 0, or a HIP error code.  Allocates and frees its own buffers.
 */
int aesmi_probe_run(int kind, uint32_t iters, int reps, double *ms, double *rate,
                    double *sclk_ghz)
{
    int dev = 0, cu = 0, wall_khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess)
        return (int)e;
    if (kind < 0 || kind > 2 || reps < 1 || iters == 0)
        return (int)hipErrorInvalidValue;
    const uint32_t threads = 1024;
    const uint32_t grid = (uint32_t)cu * (kind == 2 ? 2u : 1u);
    uint64_t *clk = nullptr;
    uint32_t *sink = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    e = hipMalloc(&clk, sizeof(uint64_t) * 4 * grid);
    if (e == hipSuccess)
        e = hipMalloc(&sink, sizeof(uint32_t) * threads * grid);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    std::vector<uint64_t> h(4 * (size_t)grid);
    double cyc = 0, real = 0;
    for (int r = 0; e == hipSuccess && r <= reps; ++r) {
        if (r == 1)
            e = hipEventRecord(a, s);
        if (e != hipSuccess)
            break;
        if (kind == 0)
            hipLaunchKernelGGL(lds_probe_kernel, dim3(grid), dim3(threads), 0, s, iters, clk, sink);
        else if (kind == 1)
            hipLaunchKernelGGL(round_probe_kernel, dim3(grid), dim3(threads), 0, s, iters, clk,
                               sink);
        else
            hipLaunchKernelGGL(valu_probe_kernel, dim3(grid), dim3(threads), 0, s, iters, clk,
                               sink);
        e = hipGetLastError();
        if (e == hipSuccess && r == reps)
            e = hipEventRecord(b, s);
        if (e == hipSuccess && r == reps)
            e = hipMemcpyAsync(h.data(), clk, sizeof(uint64_t) * h.size(), hipMemcpyDeviceToHost,
                               s);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    float t = 0;
    if (e == hipSuccess)
        e = hipEventElapsedTime(&t, a, b);
    if (e == hipSuccess) {
        for (uint32_t g = 0; g < grid; ++g) {
            cyc += (double)(h[4 * g + 2] - h[4 * g]);
            real += (double)(h[4 * g + 3] - h[4 * g + 1]);
        }
        const double per = (double)t / reps;
        const double n = (double)grid * threads * iters;
        const double ops = kind == 0 ? n * kChains : kind == 1 ? n * 4 : n * kChains * 2;
        *ms = per;
        *rate = ops / (per * 1e-3);
        *sclk_ghz = real > 0 && wall_khz > 0 ? cyc / real * (double)wall_khz * 1e-6 : 0.0;
    }
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    if (s)
        (void)hipStreamDestroy(s);
    (void)hipFree(clk);
    (void)hipFree(sink);
    return (int)e;
}

}  // extern "C"
