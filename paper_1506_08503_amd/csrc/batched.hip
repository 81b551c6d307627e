// batched.hip -- placeholder until the batched kernel lands.
#include "internal.hpp"
namespace aesmi {
size_t batched_workspace_bytes(uint32_t nsegs) { return 256 + 8 * (size_t)nsegs; }
hipError_t batched_ctr(const aes_segment_t *, uint32_t, const aes_key_schedule_t *, uint32_t,
                       const uint8_t *, uint8_t *, const aes_batch_tune_t *, void *, hipStream_t)
{
    return hipErrorNotSupported;
}
}  // namespace aesmi
