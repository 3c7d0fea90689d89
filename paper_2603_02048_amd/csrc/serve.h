// serve.h -- serving loop of libhaze.so (internal).
#pragma once

#include "haze.h"
#include "haze_device.h"

#include <hip/hip_runtime.h>

namespace haze {
struct Server;
void server_destroy(Server *s);
bool server_waiting_use(hz_ctx *c, const hz_field *f, const hz_mesh *m);   // a queued request reads f or m

// context/field accessors implemented in runtime.hip
hz_status ctx_alloc(hz_ctx *c, void **p, size_t bytes);
hz_status ctx_alloc_nowait(hz_ctx *c, void **p, size_t bytes);   // no pool trimming, no device waits
void ctx_free(hz_ctx *c, void *p, size_t bytes);
void ctx_trim_pool(hz_ctx *c, size_t bytes);   // waits for the device: never under the server lock
int ctx_device(const hz_ctx *c);
int ctx_num_cus(const hz_ctx *c);
uint64_t ctx_mem_avail(const hz_ctx *c);
Server *&ctx_server(hz_ctx *c);
const hz_grid &field_grid(const hz_field *f);
hz_dtype field_dtype(const hz_field *f);
float field_scale(const hz_field *f);
const void *field_data(const hz_field *f);
hz_ctx *field_ctx(const hz_field *f);
hz_status field_ready(hz_field *f, hipStream_t s);       // order a read on s after the field's producer
void field_use(hz_field *f, const CallMark &t);            // a read by the call with mark t
hz_status ctx_mark(hz_ctx *c, hipStream_t s, CallMark *out);
hz_status ctx_mark_sync(hz_ctx *c, const CallMark &t);    // block the host until the call's work is done
int march_blocks(hz_ctx *c, int dt, int scene_mode);   // persistent march grid (scene mode 0, 1, 2 or 3)
// mesh accessors implemented in mesh.hip
const MeshLaunch &mesh_launch(const hz_mesh *m);
float mesh_reach(const hz_mesh *m);
hz_ctx *mesh_ctx(const hz_mesh *m);
void mesh_use(hz_mesh *m, const CallMark &t);   // a read by the call with mark t
void profile_add(hz_ctx *c, const char *name, double ms);
hz_status set_error(hz_status s, const char *msg);
hz_status field_usable(hz_ctx *c, const hz_field *f, const char *fn);   // pending device faults, bad fields
}  // namespace haze
