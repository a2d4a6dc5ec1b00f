// Nearest-particle statistics (section "Nearest particle statistics").
//
// For every drop i the minimum-image vectors to all other drops are formed
// exactly as in the definition (per axis: subtract L if r > L/2, add L if
// r <= -L/2; d2 = (rx^2 + ry^2) + rz^2); the nearest set is every j with d2
// equal to the minimum, with tie weight h = 1/N_i (eq. 4). Each nearest pair
// is binned in (r, theta) (eqs. 8 and 10) with integer weights 720720/N_i,
// accumulated by 64-bit integer atomics (order-independent, exact), and
// contributes h r and h r r^T to the moments M (eq. 11) and R (eq. 14).
// Per-drop moment contributions are summed in a fixed tree order, so every
// output is reproducible bit for bit.
#include <mutex>

#include "common.hpp"

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kFixedOne = 720720ull;  // lcm(1..16)
constexpr int32_t kMaxSlices = 64;          // candidate slices of the nearest search

struct Box {
  double L[3];
};

__device__ __forceinline__ double min_image(double d, double L) {
  if (d > 0.5 * L) d -= L;
  else if (d <= -0.5 * L) d += L;
  return d;
}

// Candidate slices: the j range is cut into `ns` slices of `len` indices
// (a multiple of kBlock); workgroup (ib, s) scans slice s for the kBlock
// drops of block ib and keeps, per drop, the slice's smallest d2, the first j
// attaining it and how many j attain it.
__global__ __launch_bounds__(kBlock) void k_nearest_slice(const double *__restrict__ xyz, int32_t n, Box box,
                                                          int32_t len, double *__restrict__ sbest,
                                                          int32_t *__restrict__ sbj, int32_t *__restrict__ sties) {
  __shared__ double sx[kBlock], sy[kBlock], sz[kBlock];
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  const int32_t s = blockIdx.y;
  double xi = 0, yi = 0, zi = 0;
  if (i < n) {
    xi = xyz[3 * (int64_t)i];
    yi = xyz[3 * (int64_t)i + 1];
    zi = xyz[3 * (int64_t)i + 2];
  }
  double best = INFINITY;
  int32_t bj = -1, ties = 0;
  const int32_t jbeg = s * len;
  const int32_t jend = (n - jbeg < len) ? n : jbeg + len;
  for (int32_t j0 = jbeg; j0 < jend; j0 += kBlock) {
    const int32_t jj = j0 + threadIdx.x;
    __syncthreads();
    if (jj < jend) {
      sx[threadIdx.x] = xyz[3 * (int64_t)jj];
      sy[threadIdx.x] = xyz[3 * (int64_t)jj + 1];
      sz[threadIdx.x] = xyz[3 * (int64_t)jj + 2];
    }
    __syncthreads();
    const int32_t m = (jend - j0 < kBlock) ? jend - j0 : kBlock;
    if (i < n) {
      for (int k = 0; k < m; ++k) {
        const int32_t j = j0 + k;
        if (j == i) continue;
        const double rx = min_image(sx[k] - xi, box.L[0]);
        const double ry = min_image(sy[k] - yi, box.L[1]);
        const double rz = min_image(sz[k] - zi, box.L[2]);
        const double d2 = (rx * rx + ry * ry) + rz * rz;
        if (d2 < best) {
          best = d2;
          bj = j;
          ties = 1;
        } else if (d2 == best) {
          ties += 1;
        }
      }
    }
  }
  if (i < n) {
    const int64_t o = (int64_t)s * n + i;
    sbest[o] = best;
    sbj[o] = bj;
    sties[o] = ties;
  }
}

// Slices combined in increasing order: the minimum over slices, the first j
// of the first slice that attains it, and the tie counts of every slice that
// attains it, which is exactly what one scan over all j in order yields.
__global__ __launch_bounds__(kBlock) void k_nearest_combine(int32_t n, int32_t ns, const double *__restrict__ sbest,
                                                            const int32_t *__restrict__ sbj,
                                                            const int32_t *__restrict__ sties,
                                                            int32_t *__restrict__ nn_index,
                                                            int32_t *__restrict__ nn_ties,
                                                            double *__restrict__ best_d2) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double best = INFINITY;
  int32_t bj = -1, ties = 0;
  for (int32_t s = 0; s < ns; ++s) {
    const int64_t o = (int64_t)s * n + i;
    const double d2 = sbest[o];
    if (d2 < best) {
      best = d2;
      bj = sbj[o];
      ties = sties[o];
    } else if (d2 == best && sties[o] > 0) {
      ties += sties[o];
    }
  }
  nn_index[i] = bj;
  nn_ties[i] = ties;
  best_d2[i] = best;
}

// Bin the nearest pairs of drop i and write its moment contributions
// part[12*i ..]: sum_j h r (3) and sum_j h r r^T (9), j ascending.
__global__ __launch_bounds__(kBlock) void k_pairs(const double *__restrict__ xyz, int32_t n, Box box, int vaxis,
                                                  int nr, int nth, const double *__restrict__ edges,
                                                  const int32_t *__restrict__ nn_index,
                                                  const int32_t *__restrict__ nn_ties,
                                                  const double *__restrict__ best_d2, uint64_t *__restrict__ hist,
                                                  double *__restrict__ part) {
  const int32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double *r2e = edges;           // nr + 1
  const double *ce = edges + nr + 1;   // nth + 1
  const double xi = xyz[3 * (int64_t)i], yi = xyz[3 * (int64_t)i + 1], zi = xyz[3 * (int64_t)i + 2];
  const double best = best_d2[i];
  const int ties = nn_ties[i];
  const double h = 1.0 / (double)ties;
  const uint64_t wfix = kFixedOne / (uint64_t)ties;
  double sm[3] = {0, 0, 0}, sr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  // No j before the first nearest index attains the minimum, and the scan
  // ends once all `ties` nearest drops are found: the same j, in the same
  // order, as a scan over every j.
  int found = 0;
  const int32_t jfirst = nn_index[i] < 0 ? 0 : nn_index[i];
  for (int32_t j = jfirst; j < n && found < ties; ++j) {
    if (j == i) continue;
    double r[3];
    r[0] = min_image(xyz[3 * (int64_t)j] - xi, box.L[0]);
    r[1] = min_image(xyz[3 * (int64_t)j + 1] - yi, box.L[1]);
    r[2] = min_image(xyz[3 * (int64_t)j + 2] - zi, box.L[2]);
    const double d2 = (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2];
    if (d2 != best) continue;
    ++found;
    int k = -1;
    for (int e = 0; e <= nr; ++e)
      if (r2e[e] <= d2) k = e;
    int m = 0;
    const double rv = (vaxis == 0) ? r[0] : ((vaxis == 1) ? r[1] : r[2]);
    for (int e = 1; e < nth; ++e) {
      const double c = ce[e];
      if (rv * fabs(rv) <= (c * fabs(c)) * d2) m = e;
    }
    if (k < 0 || k >= nr) atomicAdd((unsigned long long *)&hist[(int64_t)nr * nth], (unsigned long long)wfix);
    else atomicAdd((unsigned long long *)&hist[(int64_t)k * nth + m], (unsigned long long)wfix);
    for (int a = 0; a < 3; ++a) {
      sm[a] += h * r[a];
      for (int b = 0; b < 3; ++b) sr[3 * a + b] += h * (r[a] * r[b]);
    }
  }
  double *o = part + 12 * (int64_t)i;
  for (int a = 0; a < 3; ++a) o[a] = sm[a];
  for (int a = 0; a < 9; ++a) o[3 + a] = sr[a];
}

// Fixed-order reduction of the per-drop contributions (one workgroup), then
// the deviatoric part A = R - (tr R / 3) delta of the second moment.
__global__ __launch_bounds__(kBlock) void k_moments(const double *__restrict__ part, int32_t n, double *__restrict__ M,
                                                    double *__restrict__ R, double *__restrict__ A) {
  __shared__ double red[12][kBlock];
  double acc[12];
  for (int a = 0; a < 12; ++a) acc[a] = 0.0;
  for (int32_t i = threadIdx.x; i < n; i += kBlock)
    for (int a = 0; a < 12; ++a) acc[a] += part[12 * (int64_t)i + a];
  for (int a = 0; a < 12; ++a) red[a][threadIdx.x] = acc[a];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int a = 0; a < 12; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) M[threadIdx.x] = red[threadIdx.x][0] / (double)n;
  if (threadIdx.x < 9) R[threadIdx.x] = red[3 + threadIdx.x][0] / (double)n;
  if (A != nullptr && threadIdx.x < 9) {
    const double r0 = red[3][0] / (double)n, r4 = red[7][0] / (double)n, r8 = red[11][0] / (double)n;
    const double tr = (r0 + r4) + r8;
    const double rv = red[3 + threadIdx.x][0] / (double)n;
    A[threadIdx.x] = (threadIdx.x % 4 == 0) ? rv - tr / 3.0 : rv;
  }
}

// Densities of the nearest-pair vector at the bin centres from an
// accumulated histogram (eqs. 8 and 10): P(r, theta) = E_km / (E 2 pi r^2
// sin(theta) dr dtheta) and P_r(r) = sum_m E_km / (E 4 pi r^2 dr), E the
// events in units of 1/720720. One thread per radial bin; edges[0..nr] are
// the radii, edges[nr+1..] the polar angles.
__global__ __launch_bounds__(kBlock) void k_pair_pdfs(int32_t nr, int32_t nth, const double *__restrict__ edges,
                                                      const uint64_t *__restrict__ hist, int64_t events,
                                                      double *__restrict__ P, double *__restrict__ Pr) {
  const int32_t k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nr) return;
  const double pi = 3.14159265358979323846;
  const double *re = edges, *te = edges + nr + 1;
  const double E = (double)events * 720720.0;
  const double rc = 0.5 * (re[k] + re[k + 1]);
  const double dr = re[k + 1] - re[k];
  uint64_t row = 0;
  for (int32_t m = 0; m < nth; ++m) {
    const double tc = 0.5 * (te[m] + te[m + 1]);
    const double dth = te[m + 1] - te[m];
    const uint64_t ek = hist[(int64_t)k * nth + m];
    row += ek;
    P[(int64_t)k * nth + m] = (double)ek / (E * (2.0 * pi * (rc * rc) * sin(tc) * dr * dth));
  }
  Pr[k] = (double)row / (E * (4.0 * pi * (rc * rc) * dr));
}

__global__ void k_zero_u64(uint64_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

}  // namespace

// Argument checks shared by both entry points (host data only).
static int check_stats_args(vofmt_ctx *ctx, const char *fn, int32_t n, const double *xyz, const double *box,
                            int32_t vertical_axis, int32_t nr, int32_t ntheta, const double *r2_edges,
                            const double *cos_edges, int32_t *nn_index, int32_t *nn_ties, uint64_t *hist_fixed,
                            double *M, double *R) {
  if (n < 2 || vertical_axis < 0 || vertical_axis > 2 || nr < 1 || ntheta < 1)
    return set_err(ctx, VOFMT_E_ARG, "%s: bad sizes (n=%d nr=%d ntheta=%d axis=%d)", fn, n, nr, ntheta,
                   vertical_axis);
  if (!xyz || !box || !r2_edges || !cos_edges || !nn_index || !nn_ties || !hist_fixed || !M || !R)
    return set_err(ctx, VOFMT_E_ARG, "%s: null pointer", fn);
  for (int a = 0; a < 3; ++a)
    if (!(box[a] > 0.0)) return set_err(ctx, VOFMT_E_ARG, "%s: box must be positive", fn);
  for (int e = 0; e < nr; ++e)
    if (!(r2_edges[e] < r2_edges[e + 1])) return set_err(ctx, VOFMT_E_ARG, "%s: r2_edges must increase", fn);
  for (int e = 0; e < ntheta; ++e)
    if (!(cos_edges[e] > cos_edges[e + 1])) return set_err(ctx, VOFMT_E_ARG, "%s: cos_edges must decrease", fn);
  return VOFMT_OK;
}

// Candidate slices of the nearest search: at most kMaxSlices slices, each a
// whole number of kBlock indices.
struct SliceShape {
  int32_t nblk, len, ns;
};
static SliceShape slice_shape(int32_t n) {
  SliceShape sh;
  sh.nblk = (int32_t)ceil_div(n, kBlock);
  const int32_t per = (int32_t)ceil_div(sh.nblk, kMaxSlices);
  sh.len = per * kBlock;
  sh.ns = (int32_t)ceil_div(n, sh.len);
  return sh;
}

// The kernels of one call, on device buffers: dedge (edges, already on the
// device), best [n], part [12 n], sl (ns * n * 16 bytes).
static void launch_stats(int32_t n, const double *xyz, const double *box, int32_t vertical_axis, int32_t nr,
                         int32_t ntheta, const double *dedge, double *best, double *part, char *sl,
                         int32_t *nn_index, int32_t *nn_ties, uint64_t *hist_fixed, double *M, double *R, double *A,
                         hipStream_t stream) {
  const SliceShape sh = slice_shape(n);
  double *sbest = (double *)sl;
  int32_t *sbj = (int32_t *)(sbest + (size_t)sh.ns * n);
  int32_t *sties = sbj + (size_t)sh.ns * n;
  Box b;
  for (int a = 0; a < 3; ++a) b.L[a] = box[a];
  const int64_t nh = (int64_t)nr * ntheta + 1;
  hipLaunchKernelGGL(k_zero_u64, dim3(ceil_div(nh, 256)), dim3(256), 0, stream, hist_fixed, nh);
  hipLaunchKernelGGL(k_nearest_slice, dim3(sh.nblk, sh.ns), dim3(kBlock), 0, stream, xyz, n, b, sh.len, sbest, sbj,
                     sties);
  hipLaunchKernelGGL(k_nearest_combine, dim3(sh.nblk), dim3(kBlock), 0, stream, n, sh.ns, sbest, sbj, sties,
                     nn_index, nn_ties, best);
  hipLaunchKernelGGL(k_pairs, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, stream, xyz, n, b, vertical_axis, nr,
                     ntheta, dedge, nn_index, nn_ties, best, hist_fixed, part);
  hipLaunchKernelGGL(k_moments, dim3(1), dim3(kBlock), 0, stream, part, n, M, R, A);
}

extern "C" int vofmt_nearest_pair_stats(vofmt_ctx *ctx, int32_t n, const double *xyz, const double *box,
                                        int32_t vertical_axis, int32_t nr, int32_t ntheta, const double *r2_edges,
                                        const double *cos_edges, int32_t *nn_index, int32_t *nn_ties,
                                        uint64_t *hist_fixed, double *M, double *R, double *A,
                                        hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  int rc = check_stats_args(ctx, "vofmt_nearest_pair_stats", n, xyz, box, vertical_axis, nr, ntheta, r2_edges,
                            cos_edges, nn_index, nn_ties, hist_fixed, M, R);
  if (rc) return rc;
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const size_t nedge = (size_t)nr + 1 + (size_t)ntheta + 1;
  const SliceShape sh = slice_shape(n);
  double *dedge = (double *)scratch(ctx, SLOT_MISC, sizeof(double) * nedge);
  double *best = (double *)scratch(ctx, SLOT_MISC2, sizeof(double) * (size_t)n);
  double *part = (double *)scratch(ctx, SLOT_MISC3, sizeof(double) * 12 * (size_t)n);
  char *sl = (char *)scratch(ctx, SLOT_LABEL_A, (sizeof(double) + 2 * sizeof(int32_t)) * (size_t)sh.ns * n);
  double *hstage = (double *)host_scratch(ctx, sizeof(double) * nedge);
  if (!dedge || !best || !part || !sl || !hstage) return VOFMT_E_NOMEM;
  for (int e = 0; e <= nr; ++e) hstage[e] = r2_edges[e];
  for (int e = 0; e <= ntheta; ++e) hstage[nr + 1 + e] = cos_edges[e];
  VOFMT_HIP(ctx, hipMemcpyAsync(dedge, hstage, sizeof(double) * nedge, hipMemcpyHostToDevice, stream));
  launch_stats(n, xyz, box, vertical_axis, nr, ntheta, dedge, best, part, sl, nn_index, nn_ties, hist_fixed, M, R, A,
               stream);
  VOFMT_HIP(ctx, hipGetLastError());
  // the staging buffer must stay valid until the copy has run
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  return VOFMT_OK;
}

// ---------------------------------------------------------------- no-allocation variant
//
// vofmt_nearest_pair_stats_noalloc runs the same kernels on a fixed device
// array of this file instead of context scratch, and takes the bin edges as a
// kernel argument instead of through pinned host staging, so it allocates
// nothing and does not synchronise. Limits: n <= kNoAllocMaxDrops,
// nr + ntheta + 2 <= kNoAllocMaxEdges. Every call on a device shares the
// device's copy of the array: calls that overlap on one device race.
constexpr int32_t kNoAllocMaxDrops = 8192;
constexpr int32_t kNoAllocMaxEdges = 384;
constexpr size_t kNoAllocOffBest = 256 * ((sizeof(double) * kNoAllocMaxEdges + 255) / 256);
constexpr size_t kNoAllocOffPart = kNoAllocOffBest + sizeof(double) * kNoAllocMaxDrops;
constexpr size_t kNoAllocOffSlices = kNoAllocOffPart + 12 * sizeof(double) * kNoAllocMaxDrops;
// slices of the largest call: at most ceil(8192 / kBlock) = 32 of one kBlock each
constexpr size_t kNoAllocSliceBytes = (sizeof(double) + 2 * sizeof(int32_t)) * 32 * (size_t)kNoAllocMaxDrops;
constexpr size_t kNoAllocBytes = kNoAllocOffSlices + kNoAllocSliceBytes;  // 4.8 MiB
static_assert(kNoAllocOffPart % 256 == 0 && kNoAllocOffSlices % 256 == 0, "aligned parts");
static_assert(kNoAllocMaxDrops / kBlock <= kMaxSlices, "one slice per block at the largest size");

static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDevices = 64;
static void *g_noalloc_ptr[kNoAllocMaxDevices] = {};
static std::mutex g_noalloc_mu;

// Device address of this device's copy of noalloc_scratch, looked up once per
// device with that device current (called by vofmt_create). The host-side
// name of the array is not a device address and is never passed to a kernel.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
  if (e != hipSuccess) return e;
  g_noalloc_ptr[device] = p;
  return hipSuccess;
}

struct EdgeTable {
  double e[kNoAllocMaxEdges];
};
static_assert(sizeof(EdgeTable) <= 3072, "kernel argument size");

__global__ void k_store_edges(EdgeTable t, int32_t n, double *__restrict__ out) {
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) out[i] = t.e[i];
}

extern "C" int vofmt_nearest_pair_stats_noalloc(vofmt_ctx *ctx, int32_t n, const double *xyz, const double *box,
                                                int32_t vertical_axis, int32_t nr, int32_t ntheta,
                                                const double *r2_edges, const double *cos_edges, int32_t *nn_index,
                                                int32_t *nn_ties, uint64_t *hist_fixed, double *M, double *R,
                                                double *A, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  const char *fn = "vofmt_nearest_pair_stats_noalloc";
  int rc = check_stats_args(ctx, fn, n, xyz, box, vertical_axis, nr, ntheta, r2_edges, cos_edges, nn_index, nn_ties,
                            hist_fixed, M, R);
  if (rc) return rc;
  if (n > kNoAllocMaxDrops)
    return set_err(ctx, VOFMT_E_ARG, "%s: n=%d drops exceeds the fixed scratch limit of %d", fn, n,
                   kNoAllocMaxDrops);
  if ((int64_t)nr + ntheta + 2 > kNoAllocMaxEdges)
    return set_err(ctx, VOFMT_E_ARG, "%s: nr + ntheta + 2 = %lld edges exceeds the limit of %d", fn,
                   (long long)nr + ntheta + 2, kNoAllocMaxEdges);
  const SliceShape sh = slice_shape(n);
  if ((size_t)sh.ns * n * (sizeof(double) + 2 * sizeof(int32_t)) > kNoAllocSliceBytes)
    return set_err(ctx, VOFMT_E_ARG, "%s: slice table exceeds the fixed scratch", fn);
  if (ctx->device < 0 || ctx->device >= kNoAllocMaxDevices || !g_noalloc_ptr[ctx->device])
    return set_err(ctx, VOFMT_E_HIP, "%s: the fixed scratch of device %d has no address", fn, ctx->device);
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  char *base = (char *)g_noalloc_ptr[ctx->device];
  double *dedge = (double *)base;
  double *best = (double *)(base + kNoAllocOffBest);
  double *part = (double *)(base + kNoAllocOffPart);
  char *sl = base + kNoAllocOffSlices;
  EdgeTable t;
  const int32_t ne = nr + 1 + ntheta + 1;
  for (int e = 0; e <= nr; ++e) t.e[e] = r2_edges[e];
  for (int e = 0; e <= ntheta; ++e) t.e[nr + 1 + e] = cos_edges[e];
  for (int e = ne; e < kNoAllocMaxEdges; ++e) t.e[e] = 0.0;
  hipLaunchKernelGGL(k_store_edges, dim3(1), dim3(256), 0, stream, t, ne, dedge);
  launch_stats(n, xyz, box, vertical_axis, nr, ntheta, dedge, best, part, sl, nn_index, nn_ties, hist_fixed, M, R, A,
               stream);
  VOFMT_HIP(ctx, hipGetLastError());
  return VOFMT_OK;
}

extern "C" int vofmt_pair_pdfs(vofmt_ctx *ctx, int32_t nr, int32_t ntheta, const double *r_edges,
                               const double *theta_edges, const uint64_t *hist_fixed, int64_t events, double *P,
                               double *Pr, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nr < 1 || ntheta < 1 || events < 1)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_pair_pdfs: bad sizes (nr=%d ntheta=%d events=%lld)", nr, ntheta,
                   (long long)events);
  if (!r_edges || !theta_edges || !hist_fixed || !P || !Pr)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_pair_pdfs: null pointer");
  if (!(r_edges[0] >= 0.0) || !(theta_edges[0] >= 0.0) || !(theta_edges[ntheta] <= 3.14159265358979323846))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_pair_pdfs: edges outside r >= 0, 0 <= theta <= pi");
  for (int e = 0; e < nr; ++e)
    if (!(r_edges[e] < r_edges[e + 1])) return set_err(ctx, VOFMT_E_ARG, "vofmt_pair_pdfs: r_edges must increase");
  for (int e = 0; e < ntheta; ++e)
    if (!(theta_edges[e] < theta_edges[e + 1]))
      return set_err(ctx, VOFMT_E_ARG, "vofmt_pair_pdfs: theta_edges must increase");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const size_t nedge = (size_t)nr + 1 + (size_t)ntheta + 1;
  double *dedge = (double *)scratch(ctx, SLOT_MISC, sizeof(double) * nedge);
  double *hstage = (double *)host_scratch(ctx, sizeof(double) * nedge);
  if (!dedge || !hstage) return VOFMT_E_NOMEM;
  for (int e = 0; e <= nr; ++e) hstage[e] = r_edges[e];
  for (int e = 0; e <= ntheta; ++e) hstage[nr + 1 + e] = theta_edges[e];
  VOFMT_HIP(ctx, hipMemcpyAsync(dedge, hstage, sizeof(double) * nedge, hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_pair_pdfs, dim3(ceil_div(nr, kBlock)), dim3(kBlock), 0, stream, nr, ntheta, dedge, hist_fixed,
                     events, P, Pr);
  VOFMT_HIP(ctx, hipGetLastError());
  // the staging buffer must stay valid until the copy has run
  VOFMT_HIP(ctx, hipStreamSynchronize(stream));
  return VOFMT_OK;
}
