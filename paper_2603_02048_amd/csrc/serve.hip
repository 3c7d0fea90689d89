// serve.hip -- serving loop (continuous batching of multi-view requests).
#include "serve.h"

namespace haze {
struct Server {
    int unused;
};
void server_destroy(Server *s) { delete s; }
}  // namespace haze

using namespace haze;

extern "C" hz_status hz_server_start(hz_ctx *, int32_t, int64_t)
{
    return set_error(HZ_E_UNSUPPORTED, "hz_server_start: serving not built yet");
}
extern "C" hz_status hz_submit(hz_ctx *, const hz_field *, const hz_view *, int32_t, const hz_step *, hz_ticket *)
{
    return set_error(HZ_E_UNSUPPORTED, "hz_submit: serving not built yet");
}
extern "C" hz_status hz_poll(hz_ctx *, hz_ticket, double *)
{
    return set_error(HZ_E_UNSUPPORTED, "hz_poll: serving not built yet");
}
extern "C" hz_status hz_request_outputs(hz_ctx *, hz_ticket, hz_trace_out *, int64_t *)
{
    return set_error(HZ_E_UNSUPPORTED, "hz_request_outputs: serving not built yet");
}
extern "C" hz_status hz_request_release(hz_ctx *, hz_ticket)
{
    return set_error(HZ_E_UNSUPPORTED, "hz_request_release: serving not built yet");
}
extern "C" hz_status hz_server_stop(hz_ctx *)
{
    return set_error(HZ_E_UNSUPPORTED, "hz_server_stop: serving not built yet");
}
