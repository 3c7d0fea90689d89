// serve.h -- serving loop of libhaze.so (internal).
#pragma once

#include "haze.h"
#include "haze_device.h"

#include <hip/hip_runtime.h>

namespace haze {
struct Server;
void server_destroy(Server *s);

// context/field accessors implemented in runtime.hip
hz_status ctx_alloc(hz_ctx *c, void **p, size_t bytes);
void ctx_free(hz_ctx *c, void *p, size_t bytes);
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
int march_blocks(hz_ctx *c, int dt);
KTimer profile_timer(hz_ctx *c, const char *name);
void profile_commit(hz_ctx *c, const char *name, const KTimer &t);
hz_status set_error(hz_status s, const char *msg);
}  // namespace haze
