// Batched advection: many boxes of uneven sizes and tracer counts advanced
// together. Every pass of a sweep is one persistent launch for all boxes: a
// fixed grid walks a flattened table of work items (box, tracer group, tile)
// and runs the same sweep bodies as the plain path, so each box's result is
// bit-identical to advecting it alone. The whole multi-step sequence is
// captured once into a HIP graph and replayed with a single graph launch;
// a later call with the same configuration reuses the graph.
//
// Tunables (vofmt_tuning): the marching chunk of the streaming passes and the
// persistent grid size in workgroups per compute unit; the autotuner times a
// set of candidates on copies of the fields and returns the fastest.
#include <cstring>

#include "advect_kernels.hpp"

using namespace advect;

namespace {

struct BoxDev {
  int nx, ny, nz, ntr, words;
  int xwpb;  // x-sweep: 0 whole-row wavefronts (a row's cells fit one list region), else 4 per workgroup
  Divisors dv;
  double *f[2];  // the caller's field and its ping-pong copy
  const double *s[3];
  double *fmix;
  uint64_t *bits;
  uint32_t *list[2];
  int *counts[2];
};

// A run of work items that belong to one box (and, in a streaming pass, to
// ngrp consecutive tracer groups of one size).
struct Seg {
  int64_t item0;    // first global work item of the run
  int64_t nitems;   // its length
  int box, t0;      // box, first tracer of the first group
  int64_t region0;  // first list region of the first group
  int gx, gy, gz;   // tile grid of the streaming pass (x blocks, row blocks, chunks)
  int ngrp;         // groups (group k: tracers from t0 + k * G, regions from region0 + k * gstride)
  int64_t gstride;
};

__device__ __forceinline__ int find_seg(const Seg *__restrict__ segs, int nseg, int64_t item) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// work items: wavefronts (one list region each)
__global__ __launch_bounds__(256) void k_scan_b(const BoxDev *__restrict__ boxes, const Seg *__restrict__ segs,
                                                int nseg, int64_t nitems, int rsize) {
  for (int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; gw < nitems;
       gw += (int64_t)gridDim.x * 4) {
    const Seg sg = segs[find_seg(segs, nseg, gw)];
    const BoxDev &b = boxes[sg.box];
    const int64_t total = (int64_t)b.ntr * b.nx * b.ny * b.nz;
    scan_body(b.f[0], total, b.list[0], b.counts[0], sg.nitems, rsize, gw - sg.item0);
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_plic_b(const BoxDev *__restrict__ boxes, const Seg *__restrict__ segs,
                                                int nseg, int64_t nitems, int rsize, int par, int cur) {
  for (int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; gw < nitems;
       gw += (int64_t)gridDim.x * 4) {
    const Seg sg = segs[find_seg(segs, nseg, gw)];
    const BoxDev &b = boxes[sg.box];
    plic_body<D>(b.f[par], b.s[D], b.list[cur], b.counts[cur], sg.nitems, rsize, b.fmix, b.nx, b.ny, b.nz, b.dv,
                 gw - sg.item0);
  }
}

// work items: 4-wavefront tiles of a streaming pass
template <int D, int G>
__global__ __launch_bounds__(256) void k_stream_b(const BoxDev *__restrict__ boxes, const Seg *__restrict__ segs,
                                                  int nseg, int64_t nitems, int chunk, int rsize, int par, int nxt,
                                                  int write_cc) {
  for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
    const Seg sg = segs[find_seg(segs, nseg, item)];
    const BoxDev &b = boxes[sg.box];
    // (the grid is a multiple of 8 workgroups, so items 8 apart share an XCD)
    const GroupTile g = group_tile(item - sg.item0, sg.gx, sg.gy, sg.gz, sg.ngrp, D == 1);
    const int t0 = sg.t0 + g.grp * G;
    const int64_t region0 = sg.region0 + g.grp * sg.gstride;
    if (D == 0 && b.xwpb == 0)  // uniform over the workgroup
      stream_body<D, G, 0>(b.f[par], b.f[par ^ 1], b.s[D], b.fmix, b.bits, write_cc, t0, b.nx, b.ny, b.nz, b.words,
                           chunk, b.list[nxt], b.counts[nxt], region0, rsize, g.bx, g.by, g.bz, sg.gx, sg.gy);
    else
      stream_body<D, G>(b.f[par], b.f[par ^ 1], b.s[D], b.fmix, b.bits, write_cc, t0, b.nx, b.ny, b.nz, b.words,
                        chunk, b.list[nxt], b.counts[nxt], region0, rsize, g.bx, g.by, g.bz, sg.gx, sg.gy);
  }
}

// result back into the caller's fields (after an odd number of sweeps)
__global__ __launch_bounds__(256) void k_copy_b(const BoxDev *__restrict__ boxes, int nboxes) {
  for (int bi = 0; bi < nboxes; ++bi) {
    const BoxDev &b = boxes[bi];
    const int64_t n = (int64_t)b.ntr * b.nx * b.ny * b.nz;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x)
      b.f[0][q] = b.f[1][q];
  }
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Plan {
  int nboxes;
  int chunk, rsize, grid;
  // table offsets in the slab (bytes) and segment counts
  size_t off_boxes;
  size_t off_scan;
  int n_scan;
  int64_t items_scan;
  size_t off_plic[3];  // list regions after a sweep along d
  int n_plic[3];
  int64_t items_plic[3];
  size_t off_stream[3][3];  // [d][group kind: 4, 2, 1]
  int n_stream[3][3];
  int64_t items_stream[3][3];
};

int kind_of(int g) { return g == 4 ? 0 : (g == 2 ? 1 : 2); }

// x-sweep layout of a box: whole-row wavefronts when a row has at most `chunk`
// segments (its cells then fit a wavefront's list region), else 4 wavefronts
// per workgroup sharing segment ends through LDS.
int box_xwpb(int words, int chunk) { return words <= chunk ? 0 : 4; }

}  // namespace

static int validate(vofmt_ctx *ctx, int32_t nboxes, const vofmt_box *boxes, const char *who) {
  if (nboxes < 0 || (nboxes > 0 && !boxes)) return set_err(ctx, VOFMT_E_ARG, "%s: bad box table", who);
  for (int i = 0; i < nboxes; ++i) {
    const vofmt_box &b = boxes[i];
    if (b.nx < 1 || b.ny < 1 || b.nz < 1 || b.ntracers < 1)
      return set_err(ctx, VOFMT_E_ARG, "%s: box %d has bad sizes", who, i);
    if (!b.c || !b.sx || !b.sy || !b.sz) return set_err(ctx, VOFMT_E_ARG, "%s: box %d has a null pointer", who, i);
    if ((int64_t)b.ntracers * b.nx * b.ny * b.nz >= ((int64_t)1 << 32))
      return set_err(ctx, VOFMT_E_ARG, "%s: box %d: ntracers * cells must stay below 2^32", who, i);
  }
  return VOFMT_OK;
}

static int resolve_tuning(vofmt_ctx *ctx, const vofmt_tuning *tuning, int *chunk, int *wg_per_cu) {
  *chunk = 32;
  *wg_per_cu = 8;
  if (tuning) {
    *chunk = tuning->chunk;
    *wg_per_cu = tuning->workgroups_per_cu;
  }
  if (!(*chunk == 8 || *chunk == 16 || *chunk == 32 || *chunk == 64) || *wg_per_cu < 1 || *wg_per_cu > 32)
    return set_err(ctx, VOFMT_E_ARG, "vofmt tuning: chunk must be 8, 16, 32 or 64 and workgroups_per_cu 1..32");
  return VOFMT_OK;
}

// Lay out the slab (per-box buffers, then the tables) and fill the host copy
// of the tables. Returns the slab size in bytes.
static size_t plan_layout(const vofmt_box *boxes, int nboxes, int chunk, Plan &pl, std::vector<BoxDev> &bd,
                          std::vector<Seg> &seg_all, std::vector<size_t> &box_off) {
  const int rsize = region_size(chunk);
  pl.nboxes = nboxes;
  pl.chunk = chunk;
  pl.rsize = rsize;
  size_t off = 0;
  bd.assign(nboxes, BoxDev{});
  box_off.assign(nboxes * 6, 0);
  for (int i = 0; i < nboxes; ++i) {
    const vofmt_box &b = boxes[i];
    const int64_t n3 = (int64_t)b.nx * b.ny * b.nz;
    const int words = (int)ceil_div(b.nx, 64);
    const int xw = box_xwpb(words, chunk);
    const int64_t maxreg = max_regions(b.nx, b.ny, b.nz, b.ntracers, chunk, xw);
    const size_t field = sizeof(double) * (size_t)n3 * b.ntracers;
    box_off[6 * i + 0] = off;  // ping-pong field
    off = align256(off + field);
    box_off[6 * i + 1] = off;  // fmix
    off = align256(off + field);
    box_off[6 * i + 2] = off;  // c > 0.5 bits
    off = align256(off + sizeof(uint64_t) * (size_t)b.ntracers * b.nz * b.ny * words);
    box_off[6 * i + 3] = off;  // two lists
    off = align256(off + sizeof(uint32_t) * 2 * (size_t)maxreg * rsize);
    box_off[6 * i + 4] = off;  // two count arrays
    off = align256(off + sizeof(int) * 2 * (size_t)maxreg);
    box_off[6 * i + 5] = (size_t)maxreg;
    BoxDev &d = bd[i];
    d.nx = b.nx;
    d.ny = b.ny;
    d.nz = b.nz;
    d.ntr = b.ntracers;
    d.words = words;
    d.xwpb = xw;
    d.dv.n3 = make_fastdiv((uint32_t)n3);
    d.dv.nx = make_fastdiv((uint32_t)b.nx);
    d.dv.ny = make_fastdiv((uint32_t)b.ny);
    d.s[0] = b.sx;
    d.s[1] = b.sy;
    d.s[2] = b.sz;
  }
  // segment tables
  seg_all.clear();
  auto begin_table = [&](size_t &table_off, int &n, int64_t &items) {
    table_off = seg_all.size();
    n = 0;
    items = 0;
  };
  // initial scan: regions of rsize tracer-cells
  begin_table(pl.off_scan, pl.n_scan, pl.items_scan);
  for (int i = 0; i < nboxes; ++i) {
    const int64_t total = (int64_t)boxes[i].ntracers * boxes[i].nx * boxes[i].ny * boxes[i].nz;
    Seg s{};
    s.item0 = pl.items_scan;
    s.nitems = (total + rsize - 1) / rsize;
    s.box = i;
    seg_all.push_back(s);
    pl.items_scan += s.nitems;
    ++pl.n_scan;
  }
  for (int d = 0; d < 3; ++d) {
    begin_table(pl.off_plic[d], pl.n_plic[d], pl.items_plic[d]);
    for (int i = 0; i < nboxes; ++i) {
      const vofmt_box &b = boxes[i];
      Seg s{};
      s.item0 = pl.items_plic[d];
      const int xw = box_xwpb((b.nx + 63) / 64, chunk);
      s.nitems = stream_waves(d, b.nx, b.ny, b.nz, chunk, xw) * num_groups(b.ntracers);
      s.box = i;
      seg_all.push_back(s);
      pl.items_plic[d] += s.nitems;
      ++pl.n_plic[d];
    }
  }
  for (int d = 0; d < 3; ++d)
    for (int kind = 0; kind < 3; ++kind) {
      begin_table(pl.off_stream[d][kind], pl.n_stream[d][kind], pl.items_stream[d][kind]);
      for (int i = 0; i < nboxes; ++i) {
        const vofmt_box &b = boxes[i];
        const int xw = box_xwpb((b.nx + 63) / 64, chunk);
        const Tiles tg = stream_tiles(d, b.nx, b.ny, b.nz, chunk, xw);
        const int gx = tg.gx, gy = tg.gy, gz = tg.gz;
        const int64_t per = stream_waves(d, b.nx, b.ny, b.nz, chunk, xw);
        // all full groups of the box in one run of items, then one run per
        // group of 2 or 1 (list regions in group order, as in the plain path)
        const int nfull = b.ntracers / kMaxGroup;
        int64_t region0 = 0;
        for (int t = 0; t < b.ntracers;) {
          const int g = group_size(b.ntracers - t);
          const int ng = (g == kMaxGroup) ? nfull : 1;
          if (kind_of(g) == kind) {
            Seg s{};
            s.item0 = pl.items_stream[d][kind];
            s.nitems = (int64_t)gx * gy * gz * ng;
            s.box = i;
            s.t0 = t;
            s.region0 = region0;
            s.gx = gx;
            s.gy = gy;
            s.gz = gz;
            s.ngrp = ng;
            s.gstride = per;
            seg_all.push_back(s);
            pl.items_stream[d][kind] += s.nitems;
            ++pl.n_stream[d][kind];
          }
          t += g * ng;
          region0 += per * ng;
        }
      }
    }
  // tables after the per-box buffers: boxes, then segments
  pl.off_boxes = off;
  off = align256(off + sizeof(BoxDev) * (size_t)(nboxes > 0 ? nboxes : 1));
  const size_t seg_base = off;
  off = align256(off + sizeof(Seg) * (seg_all.size() > 0 ? seg_all.size() : 1));
  // convert segment indices to byte offsets
  auto to_bytes = [&](size_t idx) { return seg_base + idx * sizeof(Seg); };
  pl.off_scan = to_bytes(pl.off_scan);
  for (int d = 0; d < 3; ++d) {
    pl.off_plic[d] = to_bytes(pl.off_plic[d]);
    for (int k = 0; k < 3; ++k) pl.off_stream[d][k] = to_bytes(pl.off_stream[d][k]);
  }
  return off;
}

template <int D>
static void enqueue_sweep(uint8_t *slab, const Plan &pl, const BoxDev *dboxes, int prev_d, int par, int cur,
                          int wcc, hipStream_t st) {
  const Seg *psegs;
  int pn;
  int64_t pitems;
  if (prev_d < 0) {
    psegs = (const Seg *)(slab + pl.off_scan);
    pn = pl.n_scan;
    pitems = pl.items_scan;
  } else {
    psegs = (const Seg *)(slab + pl.off_plic[prev_d]);
    pn = pl.n_plic[prev_d];
    pitems = pl.items_plic[prev_d];
  }
  hipLaunchKernelGGL((k_plic_b<D>), dim3(pl.grid), dim3(256), 0, st, dboxes, psegs, pn, pitems, pl.rsize, par, cur);
  for (int kind = 0; kind < 3; ++kind) {
    if (pl.n_stream[D][kind] == 0) continue;
    const Seg *ss = (const Seg *)(slab + pl.off_stream[D][kind]);
    const int n = pl.n_stream[D][kind];
    const int64_t it = pl.items_stream[D][kind];
    if (kind == 0)
      hipLaunchKernelGGL((k_stream_b<D, 4>), dim3(pl.grid), dim3(256), 0, st, dboxes, ss, n, it, pl.chunk, pl.rsize,
                         par, cur ^ 1, wcc);
    else if (kind == 1)
      hipLaunchKernelGGL((k_stream_b<D, 2>), dim3(pl.grid), dim3(256), 0, st, dboxes, ss, n, it, pl.chunk, pl.rsize,
                         par, cur ^ 1, wcc);
    else
      hipLaunchKernelGGL((k_stream_b<D, 1>), dim3(pl.grid), dim3(256), 0, st, dboxes, ss, n, it, pl.chunk, pl.rsize,
                         par, cur ^ 1, wcc);
  }
}

extern "C" int vofmt_advect_batched(vofmt_ctx *ctx, int32_t nboxes, const vofmt_box *boxes, int64_t step0,
                                    int32_t nsteps, const vofmt_tuning *tuning, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nsteps < 0 || step0 < 0) return set_err(ctx, VOFMT_E_ARG, "vofmt_advect_batched: bad step range");
  int rc = validate(ctx, nboxes, boxes, "vofmt_advect_batched");
  if (rc) return rc;
  int chunk, wg;
  rc = resolve_tuning(ctx, tuning, &chunk, &wg);
  if (rc) return rc;
  if (nboxes == 0 || nsteps == 0) return VOFMT_OK;
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  Plan pl;
  std::vector<BoxDev> bd;
  std::vector<Seg> segs;
  std::vector<size_t> boff;
  const size_t bytes = plan_layout(boxes, nboxes, chunk, pl, bd, segs, boff);
  uint8_t *slab = (uint8_t *)scratch(ctx, SLOT_BATCH, bytes);
  if (!slab) return VOFMT_E_NOMEM;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  pl.grid = cus * wg;
  for (int i = 0; i < nboxes; ++i) {
    BoxDev &d = bd[i];
    d.f[0] = boxes[i].c;
    d.f[1] = (double *)(slab + boff[6 * i + 0]);
    d.fmix = (double *)(slab + boff[6 * i + 1]);
    d.bits = (uint64_t *)(slab + boff[6 * i + 2]);
    const size_t maxreg = boff[6 * i + 5];
    d.list[0] = (uint32_t *)(slab + boff[6 * i + 3]);
    d.list[1] = d.list[0] + maxreg * pl.rsize;
    d.counts[0] = (int *)(slab + boff[6 * i + 4]);
    d.counts[1] = d.counts[0] + maxreg;
  }
  // the key of this configuration: boxes, tuning, sweep order, slab
  std::string key;
  key.append((const char *)boxes, sizeof(vofmt_box) * (size_t)nboxes);
  const int64_t hdr[5] = {step0 % 3, nsteps, chunk, wg, (int64_t)(uintptr_t)slab};
  key.append((const char *)hdr, sizeof(hdr));
  if (ctx->graph && ctx->graph_key == key) {
    VOFMT_HIP(ctx, hipGraphLaunch(ctx->graph, stream));
    return VOFMT_OK;
  }
  if (ctx->graph) {
    VOFMT_HIP(ctx, hipDeviceSynchronize());  // the old graph may still run, on any stream
    (void)hipGraphExecDestroy(ctx->graph);
    ctx->graph = nullptr;
    ctx->graph_key.clear();
  }
  // tables: host copy kept in the context until the next rebuild
  const size_t tab0 = pl.off_boxes;
  ctx->tables.assign(bytes - tab0, 0);
  memcpy(ctx->tables.data(), bd.data(), sizeof(BoxDev) * bd.size());
  const size_t seg_base = align256(tab0 + sizeof(BoxDev) * (size_t)nboxes) - tab0;
  if (!segs.empty()) memcpy(ctx->tables.data() + seg_base, segs.data(), sizeof(Seg) * segs.size());
  VOFMT_HIP(ctx, hipMemcpyAsync(slab + tab0, ctx->tables.data(), ctx->tables.size(), hipMemcpyHostToDevice, stream));
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  if (!ctx->capture_stream) VOFMT_HIP(ctx, hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
  hipStream_t cs = ctx->capture_stream;
  const BoxDev *dboxes = (const BoxDev *)(slab + tab0);
  VOFMT_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_scan_b, dim3(pl.grid), dim3(256), 0, cs, dboxes, (const Seg *)(slab + pl.off_scan), pl.n_scan,
                     pl.items_scan, pl.rsize);
  int par = 0, cur = 0, prev_d = -1;
  for (int32_t st = 0; st < nsteps; ++st) {
    const int64_t g = step0 + st;
    for (int r = 0; r < 3; ++r) {
      const int d = (int)((g + r) % 3);
      const int wcc = (r == 0);
      if (d == 0) enqueue_sweep<0>(slab, pl, dboxes, prev_d, par, cur, wcc, cs);
      else if (d == 1) enqueue_sweep<1>(slab, pl, dboxes, prev_d, par, cur, wcc, cs);
      else enqueue_sweep<2>(slab, pl, dboxes, prev_d, par, cur, wcc, cs);
      prev_d = d;
      par ^= 1;
      cur ^= 1;
    }
  }
  if (par == 1) hipLaunchKernelGGL(k_copy_b, dim3(pl.grid), dim3(256), 0, cs, dboxes, nboxes);
  hipGraph_t graph = nullptr;
  const hipError_t launch_err = hipGetLastError();
  const hipError_t end_err = hipStreamEndCapture(cs, &graph);
  if (launch_err != hipSuccess || end_err != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return hip_check(ctx, launch_err != hipSuccess ? launch_err : end_err, "batched advection capture");
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t inst_err = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (inst_err != hipSuccess) return hip_check(ctx, inst_err, "hipGraphInstantiate");
  ctx->graph = exec;
  ctx->graph_key = key;
  VOFMT_HIP(ctx, hipGraphLaunch(ctx->graph, stream));
  return VOFMT_OK;
}

extern "C" int vofmt_autotune_batched(vofmt_ctx *ctx, int32_t nboxes, const vofmt_box *boxes, int32_t nsteps,
                                      vofmt_tuning *best_host, float *best_ms_host, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (!best_host || nsteps < 1) return set_err(ctx, VOFMT_E_ARG, "vofmt_autotune_batched: bad arguments");
  int rc = validate(ctx, nboxes, boxes, "vofmt_autotune_batched");
  if (rc) return rc;
  best_host->chunk = 32;
  best_host->workgroups_per_cu = 8;
  if (best_ms_host) *best_ms_host = 0.0f;
  if (nboxes == 0) return VOFMT_OK;
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  // copies of the fields, so that the caller's data is not advanced
  size_t total = 0;
  std::vector<size_t> off(nboxes);
  for (int i = 0; i < nboxes; ++i) {
    off[i] = total;
    total = align256(total + sizeof(double) * (size_t)boxes[i].ntracers * boxes[i].nx * boxes[i].ny * boxes[i].nz);
  }
  uint8_t *copies = (uint8_t *)scratch(ctx, SLOT_TUNE, total);
  if (!copies) return VOFMT_E_NOMEM;
  std::vector<vofmt_box> cb(boxes, boxes + nboxes);
  for (int i = 0; i < nboxes; ++i) {
    cb[i].c = (double *)(copies + off[i]);
    VOFMT_HIP(ctx, hipMemcpyAsync(cb[i].c, boxes[i].c,
                                  sizeof(double) * (size_t)boxes[i].ntracers * boxes[i].nx * boxes[i].ny * boxes[i].nz,
                                  hipMemcpyDeviceToDevice, stream));
  }
  hipEvent_t e0, e1;
  VOFMT_HIP(ctx, hipEventCreate(&e0));
  VOFMT_HIP(ctx, hipEventCreate(&e1));
  const int chunks[3] = {16, 32, 64};
  const int wgs[4] = {2, 4, 8, 16};
  float best = -1.0f;
  for (int a = 0; a < 3 && rc == VOFMT_OK; ++a)
    for (int b = 0; b < 4 && rc == VOFMT_OK; ++b) {
      vofmt_tuning t{chunks[a], wgs[b]};
      rc = vofmt_advect_batched(ctx, nboxes, cb.data(), 0, nsteps, &t, stream);  // builds the graph, warms up
      float ms_best = -1.0f;
      for (int rep = 0; rep < 2 && rc == VOFMT_OK; ++rep) {
        if (hipEventRecord(e0, stream) != hipSuccess) rc = set_err(ctx, VOFMT_E_HIP, "hipEventRecord failed");
        if (rc == VOFMT_OK) rc = vofmt_advect_batched(ctx, nboxes, cb.data(), 0, nsteps, &t, stream);
        if (rc == VOFMT_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
          rc = set_err(ctx, VOFMT_E_HIP, "autotune timing failed");
        float ms = 0.0f;
        if (rc == VOFMT_OK) (void)hipEventElapsedTime(&ms, e0, e1);
        if (rc == VOFMT_OK && (ms_best < 0.0f || ms < ms_best)) ms_best = ms;
      }
      if (rc == VOFMT_OK && (best < 0.0f || ms_best < best)) {
        best = ms_best;
        *best_host = t;
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (best_ms_host) *best_ms_host = best;
  return VOFMT_OK;
}
