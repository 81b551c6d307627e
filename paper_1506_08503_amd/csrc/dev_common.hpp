// dev_common.hpp -- small device helpers shared by the kernel headers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aesmi {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Three-input XOR in one VALU op (gfx950 v_bitop3_b32, truth table 0x96);
// gfx9 has no v_xor3_b32.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Byte swap: big-endian counter value <-> little-endian column word.
__device__ __forceinline__ uint32_t bswap32(uint32_t x)
{
    return __builtin_amdgcn_perm(x, x, 0x00010203u);
}

}  // namespace
}  // namespace aesmi
