// Request loop (aoresp_server_*): placeholder.
#include "runtime.h"

using namespace aoresp;

struct aoresp_server { int dummy; };

extern "C" {
aoresp_status aoresp_server_create(const aoresp_server_cfg*, aoresp_server**) { return AORESP_EINVAL; }
aoresp_status aoresp_submit(aoresp_server*, const float*, const float*, size_t, const aoresp_params*, uint64_t*) {
    return AORESP_EINVAL;
}
aoresp_status aoresp_poll(aoresp_server*, uint64_t, aoresp_result*, uint8_t*, int64_t) { return AORESP_EINVAL; }
aoresp_status aoresp_server_stats(aoresp_server*, double*, double*, double*, uint64_t*) { return AORESP_EINVAL; }
void aoresp_server_destroy(aoresp_server*) {}
}
