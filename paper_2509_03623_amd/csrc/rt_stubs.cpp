// rt_stubs.cpp -- entry points whose kernels are not in this build yet.
#include "rt_host.h"

namespace rt {
rt_status render_cube_mlp(const rt_problem *, float *, hipStream_t) {
    return fail(RT_EINVAL, "neural CO layer not available in this build");
}
rt_status adjoint_mlp(const rt_problem *, const float *, const rt_grads *, float *, hipStream_t) {
    return fail(RT_EINVAL, "neural CO layer not available in this build");
}
} // namespace rt

using namespace rt;
extern "C" {
rt_status rt_server_create(const rt_server_cfg *, rt_server **) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_submit(rt_server *, const rt_request *, uint64_t *) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_poll(rt_server *, uint64_t, rt_ticket_info *) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_wait(rt_server *, uint64_t, rt_ticket_info *, uint64_t) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_cancel(rt_server *, uint64_t) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_server_destroy(rt_server *) { return fail(RT_EINVAL, "server not available"); }
}
