// Direction-split geometric PLIC advection of N tracer fields (eq. 3 of the
// paper applied to every tracer C_i; its discrete form is the conservative
// split scheme of Weymouth & Yue 2010 with MYC normals).
//
// One launch performs one sweep along axis D for every tracer. A wavefront
// owns 64 consecutive x-cells of one row, so every load and store of a field
// row is a coalesced 512-byte transaction, and the c > 0.5 indicator of the
// 64 cells is one 64-bit ballot word. Each thread keeps its two face Courant
// numbers in registers and loops over the tracers, so the velocity is read
// from memory once per sweep for all N tracers. Pure donors (c <= 0 or
// c >= 1) cost a multiply; mixed donors take the PLIC path (3x3x3 gather,
// MYC normal, plane constant, sub-box volume).
#include "common.hpp"
#include "plic.hpp"

namespace {

constexpr int kRows = 4;  // rows of 64 cells per block (4 wavefronts)

// Phase volume fraction of the donor's upwind sub-box for a mixed donor
// (0 < cd < 1) at (i,j,k): the donor's PLIC plane {m.x <= alpha} restricted
// to x_D in [x0, x0 + |s|], mapped affinely onto the unit cube.
template <int D>
__device__ __noinline__ double mixed_subbox_fraction(const double *__restrict__ c, int i, int j, int k, int nx,
                                                     int ny, int nz, double cd, double s, double x0) {
  const int im = wrap_dec(i, nx), ip = wrap_inc(i, nx);
  const int jm = wrap_dec(j, ny), jp = wrap_inc(j, ny);
  const int km = wrap_dec(k, nz), kp = wrap_inc(k, nz);
  const int xs[3] = {im, i, ip};
  const int ys[3] = {jm, j, jp};
  const int zs[3] = {km, k, kp};
  double b[27];
#pragma unroll
  for (int az = 0; az < 3; ++az)
#pragma unroll
    for (int ay = 0; ay < 3; ++ay) {
      const double *row = c + ((int64_t)zs[az] * ny + ys[ay]) * nx;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) b[ax + 3 * ay + 9 * az] = row[xs[ax]];
    }
  double mx, my, mz;
  plic::myc_normal(b, mx, my, mz);
  double alpha = plic::alpha_of(mx, my, mz, cd);
  double md = (D == 0) ? mx : ((D == 1) ? my : mz);
  double as = alpha - md * x0;
  double ms = md * fabs(s);
  if (D == 0) return plic::volume(ms, my, mz, as);
  if (D == 1) return plic::volume(mx, ms, mz, as);
  return plic::volume(mx, my, ms, as);
}

// Flux through the face between cell a (lower along D) and cell b (upper).
template <int D>
__device__ __forceinline__ double face_flux(const double *__restrict__ c, double ca, double cb, int ai, int aj, int ak,
                                            int bi, int bj, int bk, double s, int nx, int ny, int nz) {
  if (s == 0.0) return 0.0;
  const bool up = s > 0.0;
  const double cd = up ? ca : cb;
  if (!(cd > 0.0 && cd < 1.0)) return s * cd;
  const double x0 = up ? 1.0 - s : 0.0;
  const int di = up ? ai : bi, dj = up ? aj : bj, dk = up ? ak : bk;
  return s * mixed_subbox_fraction<D>(c, di, dj, dk, nx, ny, nz, cd, s, x0);
}

template <int D>
__global__ __launch_bounds__(64 * kRows) void k_sweep(const double *__restrict__ cin, double *__restrict__ cout,
                                                      const double *__restrict__ s, uint64_t *__restrict__ ccbits,
                                                      int write_cc, int nx, int ny, int nz, int ntr, int words) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * kRows + threadIdx.y;
  const int k = blockIdx.z;
  const bool live = (i < nx) && (j < ny);
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int lane = threadIdx.x;  // 0..63 within the wavefront
  const int64_t wrow = ((int64_t)k * ny + (live ? j : 0)) * words + blockIdx.x;  // word of this row segment

  int ia = i, ja = j, ka = k, ib = i, jb = j, kb = k;  // neighbours along D: a = p - e_D, b = p + e_D
  int64_t p = 0, pa = 0, pb = 0;
  double s_lo = 0.0, s_hi = 0.0;
  if (live) {
    if (D == 0) { ia = wrap_dec(i, nx); ib = wrap_inc(i, nx); }
    if (D == 1) { ja = wrap_dec(j, ny); jb = wrap_inc(j, ny); }
    if (D == 2) { ka = wrap_dec(k, nz); kb = wrap_inc(k, nz); }
    p = ((int64_t)k * ny + j) * nx + i;
    pa = ((int64_t)ka * ny + ja) * nx + ia;
    pb = ((int64_t)kb * ny + jb) * nx + ib;
    s_lo = s[p];
    s_hi = s[pb];
  }
  for (int t = 0; t < ntr; ++t) {
    const double *ct = cin + (int64_t)t * n3;
    double c0 = 0.0, cm = 0.0, cp = 0.0;
    if (live) {
      c0 = ct[p];
      cm = ct[pa];
      cp = ct[pb];
    }
    uint64_t *bits = ccbits + (int64_t)t * nz * ny * words;
    double ccv;
    if (write_cc) {
      const uint64_t word = __ballot(live && c0 > 0.5);
      if (lane == 0 && live) bits[wrow] = word;
      ccv = (live && c0 > 0.5) ? 1.0 : 0.0;
    } else {
      const uint64_t word = live ? bits[wrow] : 0ull;
      ccv = ((word >> lane) & 1ull) ? 1.0 : 0.0;
    }
    if (!live) continue;
    const double f_lo = face_flux<D>(ct, cm, c0, ia, ja, ka, i, j, k, s_lo, nx, ny, nz);
    const double f_hi = face_flux<D>(ct, c0, cp, i, j, k, ib, jb, kb, s_hi, nx, ny, nz);
    cout[(int64_t)t * n3 + p] = (c0 - (f_hi - f_lo)) + ccv * (s_hi - s_lo);
  }
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

extern "C" int vofmt_advect(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, double *c,
                            const double *sx, const double *sy, const double *sz, int64_t step0, int32_t nsteps,
                            hipStream_t stream) {
  if (!ctx) return VOFMT_E_ARG;
  if (nx < 1 || ny < 1 || nz < 1 || ntracers < 0 || nsteps < 0 || step0 < 0)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: bad sizes (nx=%d ny=%d nz=%d ntracers=%d nsteps=%d step0=%lld)",
                   nx, ny, nz, ntracers, nsteps, (long long)step0);
  if (ntracers == 0 || nsteps == 0) return VOFMT_OK;
  if (!c || !sx || !sy || !sz) return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: null pointer");
  if ((int64_t)ny * nz > (int64_t)65535 * kRows * 65535)
    return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: grid too large");
  if (nz > 65535 || ceil_div(ny, kRows) > 65535) return set_err(ctx, VOFMT_E_ARG, "vofmt_advect: grid too large");
  VOFMT_HIP(ctx, hipSetDevice(ctx->device));
  const int64_t n3 = (int64_t)nx * ny * nz;
  const int words = (int)ceil_div(nx, 64);
  double *tmp = (double *)scratch(ctx, SLOT_PINGPONG, sizeof(double) * (size_t)n3 * ntracers);
  if (!tmp) return ctx->err.empty() ? VOFMT_E_NOMEM : VOFMT_E_NOMEM;
  uint64_t *bits = (uint64_t *)scratch(ctx, SLOT_CCBITS, sizeof(uint64_t) * (size_t)ntracers * nz * ny * words);
  if (!bits) return VOFMT_E_NOMEM;
  const double *s3[3] = {sx, sy, sz};
  dim3 block(64, kRows, 1);
  dim3 grid(words, ceil_div(ny, kRows), nz);
  double *cur = c, *nxt = tmp;
  for (int32_t st = 0; st < nsteps; ++st) {
    const int64_t g = step0 + st;
    for (int r = 0; r < 3; ++r) {
      const int d = (int)((g + r) % 3);
      const int wcc = (r == 0);
      if (d == 0)
        hipLaunchKernelGGL(k_sweep<0>, grid, block, 0, stream, cur, nxt, s3[0], bits, wcc, nx, ny, nz, ntracers, words);
      else if (d == 1)
        hipLaunchKernelGGL(k_sweep<1>, grid, block, 0, stream, cur, nxt, s3[1], bits, wcc, nx, ny, nz, ntracers, words);
      else
        hipLaunchKernelGGL(k_sweep<2>, grid, block, 0, stream, cur, nxt, s3[2], bits, wcc, nx, ny, nz, ntracers, words);
      VOFMT_HIP(ctx, hipGetLastError());
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
