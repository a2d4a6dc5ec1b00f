// Plain advection entry points: one box, one launch per pass.
// The kernels are thin wrappers around the shared sweep bodies: every sweep
// is a PLIC pass over the mixed cells and one streaming pass per tracer group.
#include "advect_kernels.hpp"

using namespace advect;

namespace {

constexpr int kChunk = 32;  // cells per thread along its marching axis
constexpr int kXWaves = 8;  // wavefronts per workgroup of the x-sweep: a 512-cell row per workgroup

__global__ __launch_bounds__(256) void k_scan_mixed(const double *__restrict__ c, int64_t total,
                                                    uint32_t *__restrict__ list, int *__restrict__ counts,
                                                    int64_t nregions, int rsize) {
  scan_body(c, total, list, counts, nregions, rsize, ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
}

template <int D>
__global__ __launch_bounds__(256) void k_plic(const double *__restrict__ cin, const double *__restrict__ s,
                                              const uint32_t *__restrict__ list, const int *__restrict__ counts,
                                              int64_t nregions, int rsize, double *__restrict__ fmix, int nx, int ny,
                                              int nz, Divisors dv) {
  plic_body<D>(cin, s, list, counts, nregions, rsize, fmix, nx, ny, nz, dv,
               ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
}

template <int D, int G>
__global__ __launch_bounds__(64 * kXWaves) void k_stream(const double *__restrict__ cin, double *__restrict__ cout,
                                                        const double *__restrict__ s, const double *__restrict__ fmix,
                                                        uint64_t *__restrict__ ccbits, int write_cc, int t0, int nx,
                                                        int ny, int nz, int words, int chunk,
                                                        uint32_t *__restrict__ list_next, int *__restrict__ counts_next,
                                                        int64_t region0, int rsize, int ngrp, int64_t gstride) {
  const GroupTile g = group_tile(((int)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x, gridDim.x,
                                 gridDim.y, gridDim.z / ngrp, ngrp, D == 1);
  stream_body<D, G, kXWaves>(cin, cout, s, fmix, ccbits, write_cc, t0 + g.grp * G, nx, ny, nz, words, chunk,
                             list_next, counts_next, region0 + g.grp * gstride, rsize, g.bx, g.by, g.bz, gridDim.x,
                             gridDim.y);
}

// The x-sweep marching along whole rows (4 wavefronts per workgroup).
template <int G>
__global__ __launch_bounds__(256) void k_stream_rows(const double *__restrict__ cin, double *__restrict__ cout,
                                                     const double *__restrict__ s, const double *__restrict__ fmix,
                                                     uint64_t *__restrict__ ccbits, int write_cc, int t0, int nx,
                                                     int ny, int nz, int words, int chunk,
                                                     uint32_t *__restrict__ list_next, int *__restrict__ counts_next,
                                                     int64_t region0, int rsize, int ngrp, int64_t gstride) {
  const GroupTile g = group_tile(((int)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x, gridDim.x,
                                 gridDim.y, gridDim.z / ngrp, ngrp, false);
  stream_body<0, G, 0>(cin, cout, s, fmix, ccbits, write_cc, t0 + g.grp * G, nx, ny, nz, words, chunk, list_next,
                       counts_next, region0 + g.grp * gstride, rsize, g.bx, g.by, g.bz, gridDim.x, gridDim.y);
}

// Per-block maximum of |s| over the three arrays and a non-finite flag.
__global__ __launch_bounds__(256) void k_courant_max(const double *__restrict__ sx, const double *__restrict__ sy,
                                                     const double *__restrict__ sz, int64_t n, double *__restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
    double a = fabs(sx[q]), b = fabs(sy[q]), c = fabs(sz[q]);
    if (!(a <= 1e300) || !(b <= 1e300) || !(c <= 1e300)) m = INFINITY;  // NaN or inf
    else m = fmax(m, fmax(a, fmax(b, c)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

}  // namespace

struct SweepBuffers {
  double *fmix;
  uint64_t *bits;
  uint32_t *list[2];
  int *counts[2];
  int64_t nregions[2];  // regions filled into each list
  int rsize;
};

static const char *stream_name(int d, int g) {
  static const char *names[3][3] = {{"k_stream<0,1>", "k_stream<0,2>", "k_stream<0,4>"},
                                    {"k_stream<1,1>", "k_stream<1,2>", "k_stream<1,4>"},
                                    {"k_stream<2,1>", "k_stream<2,2>", "k_stream<2,4>"}};
  return names[d][g == 4 ? 2 : (g == 2 ? 1 : 0)];
}

// Workgroup layout of the x-sweep: whole-row wavefronts (0) when a row has at
// most `chunk` segments (so a wavefront's cells fit its list region), else
// kXWaves wavefronts sharing segment ends through LDS.
static inline int x_wpb(int words, int chunk) { return words <= chunk ? 0 : kXWaves; }

// One streaming launch over ngrp consecutive groups of G tracers from t0;
// group k fills list regions region0 + k*per onwards.
template <int D, int G>
static void launch_stream(vofmt_ctx *ctx, const double *cin, double *cout, const double *s, SweepBuffers &sb, int wcc,
                          int t0, int ngrp, int nx, int ny, int nz, int words, int chunk, int nxt, int64_t region0,
                          int64_t per, hipStream_t stream) {
  const int wpb = (D == 0) ? x_wpb(words, chunk) : 4;
  const Tiles tg = stream_tiles(D, nx, ny, nz, chunk, wpb);
  dim3 grid(tg.gx, tg.gy, tg.gz * ngrp);
  const int rec = prof_begin(ctx, stream_name(D, G), stream);
  if (D == 0 && wpb == 0)
    hipLaunchKernelGGL((k_stream_rows<G>), grid, dim3(256), 0, stream, cin, cout, s, sb.fmix, sb.bits, wcc,
                       t0, nx, ny, nz, words, chunk,
                       sb.list[nxt], sb.counts[nxt], region0, sb.rsize, ngrp, per);
  else
    hipLaunchKernelGGL((k_stream<D, G>), grid, dim3(D == 0 ? 64 * kXWaves : 256), 0, stream, cin, cout, s,
                       sb.fmix, sb.bits, wcc, t0, nx, ny,
                       nz,
                       words, chunk, sb.list[nxt], sb.counts[nxt], region0, sb.rsize, ngrp, per);
  prof_end(ctx, rec, stream);
}

template <int D>
static void launch_sweep_axis(vofmt_ctx *ctx, const double *cin, double *cout, const double *s, SweepBuffers &sb,
                              int wcc, int cur, int nx, int ny, int nz, int ntr, int words, int chunk,
                              hipStream_t stream) {
  const int nxt = cur ^ 1;
  const int64_t nreg = sb.nregions[cur];
  Divisors dv;
  dv.n3 = make_fastdiv((uint32_t)((int64_t)nx * ny * nz));
  dv.nx = make_fastdiv((uint32_t)nx);
  dv.ny = make_fastdiv((uint32_t)ny);
  static const char *plic_names[3] = {"k_plic<0>", "k_plic<1>", "k_plic<2>"};
  const int rec = prof_begin(ctx, plic_names[D], stream);
  hipLaunchKernelGGL((k_plic<D>), dim3(ceil_div(nreg, 4)), dim3(256), 0, stream, cin, s, sb.list[cur],
                     sb.counts[cur], nreg, sb.rsize, sb.fmix, nx, ny, nz, dv);
  prof_end(ctx, rec, stream);
  const int64_t per = stream_waves(D, nx, ny, nz, chunk, D == 0 ? x_wpb(words, chunk) : 4);
  static_assert(kMaxGroup == 4, "streaming passes are instantiated for groups of 4, 2 and 1");
  // every full group of 4 in one launch, then the groups of 2 and 1 left
  const int nfull = ntr / kMaxGroup;
  int64_t region0 = 0;
  int t = 0;
  if (nfull > 0) {
    launch_stream<D, 4>(ctx, cin, cout, s, sb, wcc, 0, nfull, nx, ny, nz, words, chunk, nxt, 0, per, stream);
    t = nfull * kMaxGroup;
    region0 = nfull * per;
  }
  while (t < ntr) {
    const int g = group_size(ntr - t);
    if (g == 2) launch_stream<D, 2>(ctx, cin, cout, s, sb, wcc, t, 1, nx, ny, nz, words, chunk, nxt, region0, per, stream);
    else launch_stream<D, 1>(ctx, cin, cout, s, sb, wcc, t, 1, nx, ny, nz, words, chunk, nxt, region0, per, stream);
    t += g;
    region0 += per;
  }
  sb.nregions[nxt] = region0;
}

static int launch_sweep(vofmt_ctx *ctx, int d, const double *cin, double *cout, const double *s, SweepBuffers &sb,
                        int wcc, int cur, int nx, int ny, int nz, int ntr, int words, int chunk, hipStream_t stream) {
  if (d == 0) launch_sweep_axis<0>(ctx, cin, cout, s, sb, wcc, cur, nx, ny, nz, ntr, words, chunk, stream);
  else if (d == 1) launch_sweep_axis<1>(ctx, cin, cout, s, sb, wcc, cur, nx, ny, nz, ntr, words, chunk, stream);
  else launch_sweep_axis<2>(ctx, cin, cout, s, sb, wcc, cur, nx, ny, nz, ntr, words, chunk, stream);
  return (int)hipGetLastError();
}

extern "C" int vofmt_advect(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, double *c,
                            const double *sx, const double *sy, const double *sz, int64_t step0, int32_t nsteps,
                            hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || ntracers < 0 || nsteps < 0 || step0 < 0)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: bad sizes (nx=%d ny=%d nz=%d ntracers=%d nsteps=%d step0=%lld)",
                   nx, ny, nz, ntracers, nsteps, (long long)step0);
  if (ntracers == 0 || nsteps == 0) return VOFMT_OK;
  if (!c || !sx || !sy || !sz) return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: null pointer");
  if (ny > 65535 || ceil_div(nz, 4) > 65535 || ceil_div(ny, kChunk) > 65535 || ceil_div(nz, kChunk) > 65535)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: grid too large");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t n3 = (int64_t)nx * ny * nz;
  if ((int64_t)ntracers * n3 >= ((int64_t)1 << 32))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: ntracers * cells must stay below 2^32");
  const double *s3[3] = {sx, sy, sz};
  const int words = (int)ceil_div(nx, 64);
  const size_t field_bytes = sizeof(double) * (size_t)n3 * ntracers;
  double *tmp = (double *)scratch(ctx, SLOT_PINGPONG, field_bytes);
  double *fmix = (double *)scratch(ctx, SLOT_FMIX, field_bytes);
  uint64_t *bits = (uint64_t *)scratch(ctx, SLOT_CCBITS, sizeof(uint64_t) * (size_t)ntracers * nz * ny * words);
  // list regions: enough for the largest sweep launch set and for the initial scan
  const int rsize = region_size(kChunk);
  const int64_t maxreg = max_regions(nx, ny, nz, ntracers, kChunk, x_wpb(words, kChunk));
  const int64_t total = (int64_t)ntracers * n3;
  const int64_t scanreg = (total + rsize - 1) / rsize;
  uint32_t *lists = (uint32_t *)scratch(ctx, SLOT_MIXLIST, sizeof(uint32_t) * 2 * (size_t)maxreg * rsize);
  int *counts = (int *)scratch(ctx, SLOT_COUNTS, sizeof(int) * 2 * (size_t)maxreg);
  if (!tmp || !fmix || !bits || !lists || !counts) return VOFMT_E_NOMEM;
  SweepBuffers sb;
  sb.fmix = fmix;
  sb.bits = bits;
  sb.list[0] = lists;
  sb.list[1] = lists + (size_t)maxreg * rsize;
  sb.counts[0] = counts;
  sb.counts[1] = counts + maxreg;
  sb.nregions[0] = scanreg;
  sb.nregions[1] = 0;
  sb.rsize = rsize;
  const int chunk = kChunk;
  // mixed cells of the input field
  const int rec = prof_begin(ctx, "k_scan_mixed", stream);
  hipLaunchKernelGGL(k_scan_mixed, dim3(ceil_div(scanreg, 4)), dim3(256), 0, stream, c, total, sb.list[0],
                     sb.counts[0], scanreg, rsize);
  prof_end(ctx, rec, stream);
  VOFMT_HIP(ctx, hipGetLastError());
  int cur_list = 0;
  double *cur = c, *nxt = tmp;
  for (int32_t st = 0; st < nsteps; ++st) {
    const int64_t g = step0 + st;
    for (int r = 0; r < 3; ++r) {
      const int d = (int)((g + r) % 3);
      const int wcc = (r == 0);
      int rc = launch_sweep(ctx, d, cur, nxt, s3[d], sb, wcc, cur_list, nx, ny, nz, ntracers, words, chunk, stream);
      if (rc) return hip_check(ctx, (hipError_t)rc, "sweep launch");
      cur_list ^= 1;
      double *t = cur;
      cur = nxt;
      nxt = t;
    }
  }
  if (cur != c)
    VOFMT_HIP(ctx, hipMemcpyAsync(c, cur, sizeof(double) * (size_t)n3 * ntracers, hipMemcpyDeviceToDevice, stream));
  return VOFMT_OK;
}

extern "C" int vofmt_check_courant(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *sx,
                                   const double *sy, const double *sz, double *smax_host, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || !sx || !sy || !sz || !smax_host)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_check_courant: bad arguments");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int nblk = 1024;
  double *part = (double *)scratch(ctx, SLOT_MISC, sizeof(double) * nblk);
  double *h = (double *)host_scratch(ctx, sizeof(double) * nblk);
  if (!part || !h) return VOFMT_E_NOMEM;
  const int64_t n = (int64_t)nx * ny * nz;
  hipLaunchKernelGGL(k_courant_max, dim3(nblk), dim3(256), 0, stream, sx, sy, sz, n, part);
  VOFMT_HIP(ctx, hipGetLastError());
  VOFMT_HIP(ctx, hipMemcpyAsync(h, part, sizeof(double) * nblk, hipMemcpyDeviceToHost, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  double m = 0.0;
  for (int b = 0; b < nblk; ++b) m = fmax(m, h[b]);
  *smax_host = m;
  if (!(m <= 1e300)) return set_err(ctx, VOFMT_E_NONFINITE, "vofmt_check_courant: non-finite face velocity");
  if (m > 0.5) return set_err(ctx, VOFMT_E_CFL, "vofmt_check_courant: max |s| = %g exceeds 0.5", m);
  return VOFMT_OK;
}
