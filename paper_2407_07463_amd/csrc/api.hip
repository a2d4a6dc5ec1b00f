// Context management, error reporting and scratch memory of libvofmt.
#include <cstdarg>
#include <cstdlib>
#include <cstring>

#include "common.hpp"

int set_err(vofmt_ctx *ctx, int code, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int hip_check(vofmt_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return VOFMT_OK;
  return set_err(ctx, e == hipErrorOutOfMemory ? VOFMT_E_NOMEM : VOFMT_E_HIP, "%s: %s", what,
                 hipGetErrorString(e));
}

void *scratch(vofmt_ctx *ctx, int slot, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (ctx->cap[slot] >= bytes) return ctx->buf[slot];
  if (ctx->buf[slot]) {
    // the previous buffer may still be in use by queued work
    if (hipDeviceSynchronize() != hipSuccess) {
      set_err(ctx, VOFMT_E_HIP, "synchronise before growing scratch failed");
      return nullptr;
    }
    (void)hipFree(ctx->buf[slot]);
    ctx->buf[slot] = nullptr;
    ctx->cap[slot] = 0;
  }
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    hip_check(ctx, e, "hipMalloc(scratch)");
    return nullptr;
  }
  ctx->buf[slot] = p;
  ctx->cap[slot] = bytes;
  return p;
}

void *host_scratch(vofmt_ctx *ctx, size_t bytes) {
  if (bytes == 0) bytes = 64;
  if (ctx->host_cap >= bytes) return ctx->host;
  if (ctx->host) (void)hipHostFree(ctx->host);
  ctx->host = nullptr;
  ctx->host_cap = 0;
  void *p = nullptr;
  hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    hip_check(ctx, e, "hipHostMalloc(staging)");
    return nullptr;
  }
  ctx->host = p;
  ctx->host_cap = bytes;
  return p;
}

static hipEvent_t prof_event(vofmt_ctx *ctx) {
  if (ctx->prof_used == ctx->prof_pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ctx->prof_pool.push_back(e);
  }
  return ctx->prof_pool[ctx->prof_used++];
}

int prof_begin(vofmt_ctx *ctx, const char *name, hipStream_t stream) {
  if (!ctx->prof_on) return -1;
  hipEvent_t a = prof_event(ctx), b = prof_event(ctx);
  if (!a || !b || hipEventRecord(a, stream) != hipSuccess) return -1;
  ctx->prof.push_back(ProfRec{name, a, b});
  return (int)ctx->prof.size() - 1;
}

void prof_end(vofmt_ctx *ctx, int rec, hipStream_t stream) {
  if (rec < 0) return;
  (void)hipEventRecord(ctx->prof[rec].b, stream);
}

extern "C" int vofmt_profile_start(vofmt_ctx *ctx) {
  if (!ctx) return VOFMT_E_ARG;
  ctx->prof.clear();
  ctx->prof_used = 0;
  ctx->prof_on = true;
  return VOFMT_OK;
}

extern "C" int vofmt_profile_stop(vofmt_ctx *ctx, int32_t max_kinds, char *names, int32_t *launches,
                                  double *total_ms, int32_t *nkinds_host) {
  if (!ctx) return VOFMT_E_ARG;
  ctx->prof_on = false;
  if (max_kinds < 0 || !nkinds_host || (max_kinds > 0 && (!names || !launches || !total_ms)))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_profile_stop: bad arguments");
  int nk = 0;
  int rc = VOFMT_OK;
  std::vector<const char *> kinds;
  for (const ProfRec &r : ctx->prof) {
    if (hipEventSynchronize(r.b) != hipSuccess) {
      rc = set_err(ctx, VOFMT_E_HIP, "vofmt_profile_stop: event wait failed");
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    int k = 0;
    while (k < (int)kinds.size() && strcmp(kinds[k], r.name) != 0) ++k;
    if (k == (int)kinds.size()) kinds.push_back(r.name);
    if (k < max_kinds) {
      if (k == nk) {
        snprintf(names + 48 * k, 48, "%s", r.name);
        launches[k] = 0;
        total_ms[k] = 0.0;
        nk = k + 1;
      }
      launches[k] += 1;
      total_ms[k] += ms;
    }
  }
  *nkinds_host = (int32_t)kinds.size();
  ctx->prof.clear();
  ctx->prof_used = 0;
  return rc;
}

extern "C" int vofmt_create(vofmt_ctx **out, int device) {
  if (!out) return VOFMT_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VOFMT_E_ARG;
  if (hipSetDevice(device) != hipSuccess) return VOFMT_E_HIP;
  vofmt_ctx *ctx = new vofmt_ctx();
  ctx->device = device;
  // the fixed scratch of the no-allocation entry point: its address on this
  // device (a failure only disables that entry point, which then says so)
  if (noalloc_setup(device) != hipSuccess) (void)hipGetLastError();
  *out = ctx;
  return VOFMT_OK;
}

extern "C" void vofmt_destroy(vofmt_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  for (int i = 0; i < kNumSlots; ++i)
    if (ctx->buf[i]) (void)hipFree(ctx->buf[i]);
  if (ctx->host) (void)hipHostFree(ctx->host);
  delete ctx;
}

extern "C" const char *vofmt_last_error(const vofmt_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" const char *vofmt_version(void) { return "vofmt 0.1 gfx950"; }
