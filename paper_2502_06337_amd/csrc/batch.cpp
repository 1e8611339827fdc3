// Batched solves (est_rotation_batch): placeholder loop, replaced by the
// persistent batched launch.
#include <hip/hip_runtime.h>

#include "runtime.h"

using namespace aoresp;

extern "C" aoresp_status est_rotation_batch_dev(const float* P, const float* Q, const uint64_t* off, uint32_t batch,
                                                const aoresp_params* prm, uint32_t prm_count, aoresp_result* out,
                                                uint8_t* masks, void* hip_stream) {
    (void)P; (void)Q; (void)off; (void)batch; (void)prm; (void)prm_count; (void)out; (void)masks; (void)hip_stream;
    return AORESP_EINVAL;
}

extern "C" aoresp_status est_rotation_batch(const float* P, const float* Q, const uint64_t* off, uint32_t batch,
                                            const aoresp_params* prm, uint32_t prm_count, aoresp_result* out,
                                            uint8_t* masks) {
    (void)P; (void)Q; (void)off; (void)batch; (void)prm; (void)prm_count; (void)out; (void)masks;
    return AORESP_EINVAL;
}
