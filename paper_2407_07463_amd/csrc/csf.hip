// Multi-tracer surface-tension force on the cell faces.
//
// The force is the sum over the tracers of gamma kappa_i grad C_i, each
// curvature computed as for a single tracer (section "The no-coalescence.h
// algorithm"), here in the balanced-force face-centred form (Popinet 2018,
// referred to in section "Numerical method"): on the lower d-face of cell p,
// between m = p - e_d and p,
//   F_d[p] = gamma * sum_i phi_i (C_i[p] - C_i[m]),
// phi_i the mean of kappa_i[p] and kappa_i[m] where both are defined, the
// defined one where one is, no contribution where neither is or where C_i
// does not jump. Undefined curvature is NaN. The tracers are summed in
// increasing order, then scaled by gamma.
//
// One pass streams every tracer's C and kappa once: a wavefront holds 64
// consecutive cells of a row, a workgroup eight rows, and each thread marches
// kZC planes along z keeping the previous plane's C and kappa of its tracers
// in registers. The y neighbours of rows 1..7 come from the wavefront below
// through LDS, so only the row below the tile is read twice; the x
// neighbours are re-read through the caches. HBM reads are about 1.1 times
// the fields' size (1.3 with four-row tiles and every y neighbour re-read).
#include <cmath>

#include "common.hpp"

namespace {

constexpr int kTX = 64, kTY = 8, kZC = 16;
constexpr int kMaxGroup = 8;

// Branch-free (selects only), so that every load of a plane is issued before
// the first use.
__device__ __forceinline__ double face_term(double cp, double cm, double kp, double km) {
  const double d = cp - cm;
  const bool hp = kp == kp, hm = km == km;  // defined: not NaN
  const double phi = hp ? (hm ? (kp + km) * 0.5 : kp) : km;
  return (d == 0.0 || !(hp || hm)) ? 0.0 : phi * d;
}

// Tracers [t0, t0 + G): the running sums start from 0 (first group) or from
// the partial sums stored by the previous group, and the last group stores
// gamma times the sums. Wavefront w of a workgroup holds row by*kTY + w; the
// y-neighbour values of rows 1.. come from the wavefront below through LDS
// (one barrier per tracer, two buffers alternating by tracer), only
// wavefront 0 loads the row below the tile. Every thread takes part in every
// barrier; threads without a cell load a clamped cell and store nothing.
template <int G>
__global__ __launch_bounds__(kTX *kTY) void k_csf(const double *__restrict__ c, const double *__restrict__ kap,
                                                  int nx, int ny, int nz, int t0, double gamma, int first, int last,
                                                  double *__restrict__ fx, double *__restrict__ fy,
                                                  double *__restrict__ fz) {
  __shared__ double xc[2][kTY][kTX], xk[2][kTY][kTX];
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs in turn, so the
  // hardware id is mapped to a tile index that gives each XCD a contiguous
  // run of tiles; neighbouring tiles (whose rows are each other's halo) then
  // share an L2.
  const unsigned nwg = gridDim.x, id = blockIdx.x;
  const unsigned per = nwg / 8, rem = nwg % 8, xk8 = id % 8;
  const unsigned L = xk8 * per + (xk8 < rem ? xk8 : rem) + id / 8;
  const unsigned tx = (nx + kTX - 1) / kTX, ty = (ny + kTY - 1) / kTY;
  const unsigned bx = L % tx, by = (L / tx) % ty, bz = L / (tx * ty);
  const int lane = threadIdx.x & (kTX - 1), w = __builtin_amdgcn_readfirstlane(threadIdx.x / kTX);
  const int x = bx * kTX + lane;
  const int y = by * kTY + w;
  const bool act = x < nx && y < ny;
  const int xc_ = x < nx ? x : nx - 1, yc = y < ny ? y : ny - 1;  // clamped cell of an inactive thread
  const int z0 = bz * kZC;
  const int z1 = z0 + kZC < nz ? z0 + kZC : nz;
  const int xm = xc_ == 0 ? nx - 1 : xc_ - 1, ym = yc == 0 ? ny - 1 : yc - 1;
  const int64_t n3 = (int64_t)nx * ny * nz, plane = (int64_t)nx * ny;
  const double *ct = c + (int64_t)t0 * n3;
  const double *kt = kap + (int64_t)t0 * n3;
  double cz[G > 0 ? G : 1], kz[G > 0 ? G : 1];
  {
    const int64_t q = (int64_t)(z0 == 0 ? nz - 1 : z0 - 1) * plane + (int64_t)yc * nx + xc_;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      cz[g] = ct[g * n3 + q];
      kz[g] = kt[g * n3 + q];
    }
  }
  for (int z = z0; z < z1; ++z) {
    const int64_t row = (int64_t)z * plane + (int64_t)yc * nx;
    const int64_t p = row + xc_, pxm = row + xm, pym = (int64_t)z * plane + (int64_t)ym * nx + xc_;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (!first && act) {
      sx = fx[p];
      sy = fy[p];
      sz = fz[p];
    }
    double cp[G > 0 ? G : 1], kp[G > 0 ? G : 1], cxm[G > 0 ? G : 1], kxm[G > 0 ? G : 1], cym[G > 0 ? G : 1],
        kym[G > 0 ? G : 1];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      cp[g] = ct[g * n3 + p];
      kp[g] = kt[g * n3 + p];
      cxm[g] = ct[g * n3 + pxm];
      kxm[g] = kt[g * n3 + pxm];
      // the row below the tile: wavefront 0 only (the others read it from LDS)
      cym[g] = (w == 0) ? ct[g * n3 + pym] : 0.0;
      kym[g] = (w == 0) ? kt[g * n3 + pym] : 0.0;
    }
    // keep the plane's loads together, ahead of their first use
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int bf = g & 1;
      xc[bf][w][lane] = cp[g];
      xk[bf][w][lane] = kp[g];
      __syncthreads();
      const double cyv = (w == 0) ? cym[g] : xc[bf][w - 1][lane];
      const double kyv = (w == 0) ? kym[g] : xk[bf][w - 1][lane];
      sx += face_term(cp[g], cxm[g], kp[g], kxm[g]);
      sy += face_term(cp[g], cyv, kp[g], kyv);
      sz += face_term(cp[g], cz[g], kp[g], kz[g]);
      cz[g] = cp[g];
      kz[g] = kp[g];
    }
    if (last) {
      sx = gamma * sx;
      sy = gamma * sy;
      sz = gamma * sz;
    }
    if (act) {
      fx[p] = sx;
      fy[p] = sy;
      fz[p] = sz;
    }
  }
}

template <int G>
void launch_csf(dim3 grid, hipStream_t stream, const double *c, const double *kap, int nx, int ny, int nz, int t0,
                double gamma, int first, int last, double *fx, double *fy, double *fz) {
  hipLaunchKernelGGL(k_csf<G>, grid, dim3(kTX * kTY), 0, stream, c, kap, nx, ny, nz, t0, gamma, first, last, fx, fy,
                     fz);
}

}  // namespace

extern "C" int vofmt_csf_force(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers,
                               const double *c, const double *kappa, double gamma, double *fx, double *fy, double *fz,
                               hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || ntracers < 0) return set_err(ctx, VOFMT_E_ARG, "vofmt_csf_force: bad sizes");
  if (!std::isfinite(gamma)) return set_err(ctx, VOFMT_E_ARG, "vofmt_csf_force: gamma is not finite");
  if (!fx || !fy || !fz || (ntracers > 0 && (!c || !kappa)))
    return set_err(ctx, VOFMT_E_ARG, "vofmt_csf_force: null pointer");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t tiles = (int64_t)ceil_div(nx, kTX) * ceil_div(ny, kTY) * ceil_div(nz, kZC);
  if (tiles > INT32_MAX) return set_err(ctx, VOFMT_E_ARG, "vofmt_csf_force: grid too large");
  const dim3 grid((unsigned)tiles);
  if (ntracers == 0) {  // no interface: zero force
    launch_csf<0>(grid, stream, c, kappa, nx, ny, nz, 0, gamma, 1, 1, fx, fy, fz);
    return hip_check(ctx, hipGetLastError(), "k_csf");
  }
  for (int t0 = 0; t0 < ntracers;) {
    const int left = ntracers - t0;
    const int g = left >= kMaxGroup ? kMaxGroup : (left >= 4 ? 4 : (left >= 2 ? 2 : 1));
    const int first = t0 == 0, last = t0 + g == ntracers;
    switch (g) {
      case 8: launch_csf<8>(grid, stream, c, kappa, nx, ny, nz, t0, gamma, first, last, fx, fy, fz); break;
      case 4: launch_csf<4>(grid, stream, c, kappa, nx, ny, nz, t0, gamma, first, last, fx, fy, fz); break;
      case 2: launch_csf<2>(grid, stream, c, kappa, nx, ny, nz, t0, gamma, first, last, fx, fy, fz); break;
      default: launch_csf<1>(grid, stream, c, kappa, nx, ny, nz, t0, gamma, first, last, fx, fy, fz); break;
    }
    VOFMT_HIP(ctx, hipGetLastError());
    t0 += g;
  }
  return VOFMT_OK;
}
