// Context management, error reporting and scratch memory of libvofmt.
#include <cstdarg>
#include <cstdlib>

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

extern "C" int vofmt_create(vofmt_ctx **out, int device) {
  if (!out) return VOFMT_E_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VOFMT_E_ARG;
  if (hipSetDevice(device) != hipSuccess) return VOFMT_E_HIP;
  vofmt_ctx *ctx = new vofmt_ctx();
  ctx->device = device;
  *out = ctx;
  return VOFMT_OK;
}

extern "C" void vofmt_destroy(vofmt_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->graph) (void)hipGraphExecDestroy(ctx->graph);
  if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  for (int i = 0; i < kNumSlots; ++i)
    if (ctx->buf[i]) (void)hipFree(ctx->buf[i]);
  if (ctx->host) (void)hipHostFree(ctx->host);
  delete ctx;
}

extern "C" const char *vofmt_last_error(const vofmt_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" const char *vofmt_version(void) { return "vofmt 0.1 gfx950"; }
