// rt_server.cpp -- continuous-batching render server (placeholder entry points).
#include "rt_host.h"

using namespace rt;
extern "C" {
rt_status rt_server_create(const rt_server_cfg *, rt_server **) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_submit(rt_server *, const rt_request *, uint64_t *) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_poll(rt_server *, uint64_t, rt_ticket_info *) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_wait(rt_server *, uint64_t, rt_ticket_info *, uint64_t) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_cancel(rt_server *, uint64_t) { return fail(RT_EINVAL, "server not available"); }
rt_status rt_server_destroy(rt_server *) { return fail(RT_EINVAL, "server not available"); }
}
