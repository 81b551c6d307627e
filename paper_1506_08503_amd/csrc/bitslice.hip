// bitslice.hip -- placeholder until the bitsliced kernels land.
#include "internal.hpp"
namespace aesmi {
hipError_t bitslice_ecb(bool, const aes_key_schedule_t *, const void *, void *, uint64_t,
                        const aes_launch_t *, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t bitslice_ctr(const aes_key_schedule_t *, const uint32_t *, uint32_t, const void *,
                        void *, uint64_t, const aes_launch_t *, hipStream_t)
{
    return hipErrorNotSupported;
}
}  // namespace aesmi
