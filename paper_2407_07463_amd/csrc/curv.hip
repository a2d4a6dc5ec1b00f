// Height-function curvature of one tracer field.
//
// The paper computes the curvature kappa_i of each tracer "as for a single
// tracer" (section "The no-coalescence.h algorithm", citing Popinet's review
// of surface-tension methods). Reading: fixed 7-cell height columns
// (Cummins, Francois & Kothe 2005). For every interface cell (c more than
// 1e-12 inside (0, 1); round-off residues of pure cells are not): the MYC
// normal m orders the candidate column axes by decreasing |m_d| (ties to the
// lower axis); an axis is usable when each of the 3x3 columns has its end on
// the phase side (-sign(m_d), sign(0) = +1) full (c >= 1 - 1e-6) and its
// other end empty (c <= 1e-6); the column sums H(u, v), offsets -3..3, with
// (u, v) along the transverse axes in increasing order give
//   kappa*Delta = -[Hxx(1+Hy^2) + Hyy(1+Hx^2) - 2 Hxy Hx Hy] / (1+Hx^2+Hy^2)^{3/2},
// +2/R on a sphere of radius R cells. Every expression is evaluated in the
// written order.
#include "compact.hpp"
#include "curv_hf.hpp"

namespace {

constexpr int kBlock = 256;

// Height-function curvature of the listed cells (persistent grid).
__global__ __launch_bounds__(kBlock) void k_curv_hf_list(const double *__restrict__ c, int nx, int ny, int nz,
                                                         const int32_t *__restrict__ list,
                                                         const int32_t *__restrict__ count,
                                                         double *__restrict__ kappa, uint8_t *__restrict__ status) {
  const int n = *count;
  for (int q = blockIdx.x * kBlock + threadIdx.x; q < n; q += gridDim.x * kBlock) {
    const int64_t p = list[q];
    double k;
    uint8_t st;
    curv::hf_cell(c, p, nx, ny, nz, k, st);
    kappa[p] = k;
    status[p] = st;
  }
}

}  // namespace

// Persistent grid of the list kernels: enough workgroups to fill the chip.
int list_grid(vofmt_ctx *ctx) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || cus < 1)
    cus = 256;
  return 8 * cus;
}

extern "C" int vofmt_curvature_hf(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *c,
                                  double *kappa, uint8_t *status, hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || !c || !kappa || !status)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_curvature_hf: bad arguments");
  const int64_t n3 = (int64_t)nx * ny * nz;
  if (n3 >= INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "vofmt_curvature_hf: too many cells");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t ntiles = compact::list_tiles(n3);
  int32_t *list = (int32_t *)scratch(ctx, SLOT_CURV_LIST, sizeof(int32_t) * (size_t)n3);
  int32_t *bc = (int32_t *)scratch(ctx, SLOT_MISC, sizeof(int32_t) * (size_t)ceil_div(n3, compact::kBlock));
  int32_t *tot = (int32_t *)scratch(ctx, SLOT_CURV_COUNT, sizeof(int32_t) * (size_t)(ntiles + 1));
  uint64_t *bits = (uint64_t *)scratch(ctx, SLOT_LIST_BITS, sizeof(uint64_t) * (size_t)ceil_div(n3, 64));
  if (!list || !bc || !tot || !bits) return VOFMT_E_NOMEM;
  int rec = prof_begin(ctx, "mixed_list", stream);
  compact::launch_ordered_list(c, n3, bc, tot, list, kappa, status, bits, stream);
  prof_end(ctx, rec, stream);
  const int32_t *count = tot + ntiles;
  rec = prof_begin(ctx, "k_curv_hf_list", stream);
  hipLaunchKernelGGL(k_curv_hf_list, dim3(list_grid(ctx)), dim3(kBlock), 0, stream, c, nx, ny, nz, list, count, kappa,
                     status);
  prof_end(ctx, rec, stream);
  return hip_check(ctx, hipGetLastError(), "curvature_hf kernels");
}
