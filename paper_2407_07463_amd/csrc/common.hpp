// Shared host/device plumbing of libvofmt: the context, error reporting,
// scratch buffers and small index helpers. Kernels live in the *.hip files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "vofmt.h"

enum { kNumSlotsDecl = 27 };

// One timed launch: HIP events recorded before and after it on its stream.
struct ProfRec {
  const char *name;
  hipEvent_t a, b;
};

struct vofmt_ctx {
  int device = 0;
  std::string err;
  // Scratch buffers, grown on demand (never shrunk) and reused by later calls.
  void *buf[kNumSlotsDecl] = {};
  size_t cap[kNumSlotsDecl] = {};
  // Pinned host staging for small results read back by synchronising calls.
  void *host = nullptr;
  size_t host_cap = 0;
  // Batched advection: the captured graph of the last configuration, the
  // stream it was captured on, its key, and the host copy of its tables.
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  std::string graph_key;
  std::vector<uint8_t> tables;
  // Per-launch timing (vofmt_profile_start / vofmt_profile_stop).
  bool prof_on = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> prof_pool;
  size_t prof_used = 0;
};

// Scratch slots (one buffer per role).
enum ScratchSlot {
  SLOT_PINGPONG = 0,  // second copy of the fields during advection
  SLOT_CCBITS = 1,    // c > 0.5 bits at the start of a step
  SLOT_LABEL_A = 2,   // labelling / recolouring work arrays
  SLOT_LABEL_B = 3,
  SLOT_LABEL_C = 4,
  SLOT_MISC = 5,
  SLOT_MISC2 = 6,
  SLOT_MISC3 = 7,
  SLOT_FMIX = 8,     // fluxes of the faces with a mixed donor
  SLOT_MIXLIST = 9,  // two lists of mixed cells (input / output of a sweep)
  SLOT_COUNTS = 10,  // their lengths
  SLOT_MLP_W = 11,     // BF16 copies of the network weights
  SLOT_MLP_ACTS = 12,  // activations kept for the backward pass
  SLOT_MLP_G = 13,     // upstream gradients and per-tile losses
  SLOT_MLP_PART = 14,  // per-tile partial gradients
  SLOT_MLP_X = 15,     // canonical stencils, network outputs
  SLOT_MLP_CELL = 16,  // their cells
  SLOT_MLP_SIGN = 17,  // and orientation signs
  SLOT_BATCH = 18,     // batched advection: per-box work buffers and tables
  SLOT_TUNE = 19,      // autotuner: copies of the fields it advects
  SLOT_CURV_LIST = 20,   // curvature: list of mixed cells
  SLOT_CURV_COUNT = 21,  // its length and that of the fallback list
  SLOT_CURV_HF = 22,     // cells handed to the height-function fallback; recolouring: list predicate bits
  SLOT_RECOLOR_LIST = 23,  // recolouring: drop-boundary and shared cells
  SLOT_OCC = 24,           // recolouring, stencil mode: occupancy bits per 64-cell row segment
  SLOT_OCC_OTHERS = 25,    // and those of the other tracers
  SLOT_LIST_BITS = 26,     // interface-cell lists: one bit per cell from the counting pass
  kNumSlots = 27,
};
static_assert(kNumSlots == kNumSlotsDecl, "scratch slot count");

int set_err(vofmt_ctx *ctx, int code, const char *fmt, ...);
// Looks up the device address of the fixed scratch array of the
// no-allocation statistics entry point for `device` (current), once per device.
hipError_t noalloc_setup(int device);
int hip_check(vofmt_ctx *ctx, hipError_t e, const char *what);
// Device scratch of at least `bytes` in slot `slot`; nullptr on failure (error set).
void *scratch(vofmt_ctx *ctx, int slot, size_t bytes);
void *host_scratch(vofmt_ctx *ctx, size_t bytes);
// Timing of one launch when profiling is on: prof_begin before the launch
// (returns a record index, or -1), prof_end after it.
int prof_begin(vofmt_ctx *ctx, const char *name, hipStream_t stream);
void prof_end(vofmt_ctx *ctx, int rec, hipStream_t stream);

#define VOFMT_HIP(ctx, call)                                  \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hip_check((ctx), e_, #call); \
  } while (0)

// Device-side helpers ------------------------------------------------------

__device__ __forceinline__ int wrap_dec(int i, int n) { return i == 0 ? n - 1 : i - 1; }
__device__ __forceinline__ int wrap_inc(int i, int n) { return i == n - 1 ? 0 : i + 1; }
__device__ __forceinline__ int wrap_any(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

static inline unsigned ceil_div(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

// Division of 32-bit unsigned integers by an invariant divisor d >= 1 with a
// multiply-high, a shift and an add (Granlund & Montgomery 1994, "round-up"
// variant): exact for every n < 2^32. Built on the host, used in kernels.
struct FastDiv {
  uint32_t d, m;
  int l;
};

static inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  if (d <= 1) {
    f.m = 0;
    f.l = 0;
    return f;
  }
  int l = 0;
  while ((1ull << l) < d) ++l;  // ceil(log2 d)
  f.l = l;
  f.m = (uint32_t)((((unsigned __int128)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  return f;
}

__device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv &f) {
  if (f.d <= 1) return n;
  const uint32_t hi = __umulhi(n, f.m);
  return (hi + ((n - hi) >> 1)) >> (f.l - 1);
}
