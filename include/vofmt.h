/*
 * vofmt -- multi-tracer geometric PLIC Volume-of-Fluid on AMD MI355X (gfx950).
 *
 * C ABI of libvofmt.so. The library implements the data-parallel hot path of
 * the non-coalescing multi-tracer VoF method of Fintzi, Pierson & Popinet
 * (arXiv 2407.07463): transport of N volume-fraction fields C_i (eq. 3 applied
 * to every tracer, section "The no-coalescence.h algorithm"), labelling of the
 * drops of each tracer (the tag.h step), drop moments, reassignment of drops
 * in near contact to other tracers (Steps 1-4), nearest-particle pair
 * statistics (section "Nearest particle statistics", eqs. 4-14) and interface
 * curvature of one tracer.
 *
 * Conventions (every function):
 *   - Grids are tri-periodic, nx x ny x nz cells, x fastest: the linear index
 *     of cell (i,j,k) is p = i + nx*(j + ny*k); cell (i,j,k) occupies
 *     [i,i+1]x[j,j+1]x[k,k+1] in cell units. Several tracers are stored one
 *     after another: c[t][k][j][i], tracer stride nx*ny*nz.
 *   - Face Courant numbers s_d[p] (cells per step, |s| <= 0.5) sit on the lower
 *     d-face of cell p, same layout as one field.
 *   - Pointers are DEVICE pointers owned by the caller unless the name ends in
 *     _host. Calls enqueue work on `stream` and return without waiting, except
 *     those with _host outputs, which synchronise the stream before returning.
 *   - A context owns scratch memory only (it grows on demand and is reused);
 *     use one context per stream. Calls on one context must not overlap.
 *   - Return 0 on success or a negative VOFMT_E_* code; vofmt_last_error()
 *     then describes the failure. Argument errors are detected on the host
 *     before anything is enqueued, so an error leaves all outputs untouched.
 *   - Floating point: FP64 for volume fractions, velocities, moments and
 *     curvature; no fused multiply-add contraction is applied to any of the
 *     method's formulas.
 */
#ifndef VOFMT_H
#define VOFMT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VOFMT_OK 0
#define VOFMT_E_ARG (-1)      /* invalid argument (null pointer, bad size, bad option) */
#define VOFMT_E_CFL (-2)      /* a face Courant number exceeds 0.5 in magnitude */
#define VOFMT_E_CAPACITY (-3) /* recolouring needs more tracers than max_tracers */
#define VOFMT_E_EXTENT (-4)   /* a drop spans half the box or more along an axis */
#define VOFMT_E_NONFINITE (-5) /* non-finite input value */
#define VOFMT_E_HIP (-6)      /* a HIP runtime call failed */
#define VOFMT_E_NOMEM (-7)    /* device allocation of scratch memory failed */

typedef struct vofmt_ctx vofmt_ctx;

/* Create a context bound to HIP device `device`. *out receives the handle. */
int vofmt_create(vofmt_ctx **out, int device);
/* Release the context and its scratch memory (waits for the device first). */
void vofmt_destroy(vofmt_ctx *ctx);
/* Message of the last failed call on this context ("" if none). Owned by the context. */
const char *vofmt_last_error(const vofmt_ctx *ctx);
/* Library version string, e.g. "vofmt 0.1 gfx950". */
const char *vofmt_version(void);

/*
 * Advect every tracer field for nsteps direction-split steps, in place.
 *
 * Operation: eq. (3) dC_i/dt + u.grad C_i = 0 for each tracer C_i (section
 * "The no-coalescence.h algorithm"), discretised by geometric PLIC VoF
 * (section "Numerical method"; its discrete form is not given in the paper):
 * step g = step0 + n sweeps the axes g mod 3, (g+1) mod 3, (g+2) mod 3; each
 * sweep along d updates every cell from the pre-sweep field
 *   c'[p] = (c[p] - (F[p+e_d] - F[p])) + cc[p] * (s_d[p+e_d] - s_d[p]),
 * where cc[p] = (c[p] > 0.5) at the start of the step and F is s times the
 * phase volume fraction of the donor's upwind sub-box of width |s|: the donor
 * value itself when the donor is not mixed (mixed: more than 1e-12 inside
 * (0, 1); round-off residues of pure cells donate like pure cells), otherwise
 * the volume under the donor's PLIC plane (Mixed-Youngs-Centred normal from
 * the block with values within 1e-12 of 0 or 1 taken as 0 or 1, plane
 * constant matching the donor's c).
 *
 * c      : [ntracers][nz][ny][nx] FP64, in/out.
 * sx,sy,sz: [nz][ny][nx] FP64 face Courant numbers; the caller guarantees
 *           |s| <= 0.5 (checked only by vofmt_check_courant).
 * step0  : global index of the first step (>= 0); only g mod 3 matters.
 * Scratch: the context keeps one extra copy of c, an array of per-face
 *           fluxes of mixed donors, two lists of up to one 32-bit entry per
 *           tracer-cell and one bit per tracer-cell.
 * Errors : VOFMT_E_ARG for null pointers or non-positive sizes, or when
 *           ntracers * nx * ny * nz reaches 2^32.
 */
int vofmt_advect(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, double *c, const double *sx,
                 const double *sy, const double *sz, int64_t step0, int32_t nsteps, hipStream_t stream);

/*
 * Largest |s| over the three face-Courant arrays, written to *smax_host
 * (synchronises). Returns VOFMT_E_CFL if it exceeds 0.5, VOFMT_E_NONFINITE if
 * any value is not finite.
 */
int vofmt_check_courant(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *sx, const double *sy,
                        const double *sz, double *smax_host, hipStream_t stream);

/*
 * Label the drops of every tracer (the tag.h step of section "The
 * no-coalescence.h algorithm": one value per region bounded by interfaces).
 * Regions are the 6-connected periodic components of {c > c_eps}, numbered
 * 1..K per tracer in increasing order of their smallest linear index; 0 is
 * background. Results are bit-identical to a sequential flood fill.
 *
 * c          : [ntracers][nz][ny][nx] FP64.
 * labels     : [ntracers][nz][ny][nx] int32, output.
 * ndrops_host: [ntracers] host int32, output K per tracer (synchronises).
 */
int vofmt_label_drops(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, const double *c,
                      double c_eps, int32_t *labels, int32_t *ndrops_host, hipStream_t stream);

/*
 * Volume and periodic centroid of every drop ("The no-coalescence.h
 * algorithm": drop properties are integrals over the cells of one tag).
 * V = sum of c over the drop; with p0 the drop's first cell (smallest linear
 * index) and offsets d = p - p0 wrapped into [-n/2, n/2) per axis, the
 * centroid is (p0 + 0.5) + sum(c d)/V, wrapped into [0, n).
 *
 * labels, ndrops_host: as produced by vofmt_label_drops.
 * vol : [D] FP64 output, D = sum of ndrops_host; drops of tracer 0 first.
 * xyz : [D][3] FP64 output, in cells.
 * Errors: VOFMT_E_EXTENT (synchronises to detect it) if a drop spans n/2 or
 *         more cells along an axis; the outputs are then still written.
 */
int vofmt_drop_moments(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, const double *c,
                       const int32_t *labels, const int32_t *ndrops_host, double *vol, double *xyz,
                       hipStream_t stream);

/*
 * Shape of every drop (appendix "Deformation of the drops"): its inertia
 * tensor about the centre of mass, I = sum over the drop's cells of
 * c ((r.r) delta - r r) + (c/6) delta with r the cell centre minus the
 * centroid (periodic, wrapped into [-n/2, n/2)); the c/6 term is the cell's own
 * extent, read as filled uniformly with density c. The aspect ratio is
 * chi = sqrt(I1/I2) with I1, I2 the largest and smallest eigenvalues of I.
 * With face Courant numbers, also the drop's mean velocity sum(c u)/sum(c),
 * u the mean of each cell's two face values per axis, in cells per step.
 *
 * labels, ndrops_host: as produced by vofmt_label_drops.
 * sx, sy, sz: [nz][ny][nx] FP64 face Courant numbers (lower faces), or all
 *             NULL together with vel.
 * inertia   : [D][6] FP64 output (Ixx, Iyy, Izz, Ixy, Ixz, Iyz), in cells^5
 *             (volume in cells^3 times length^2); drops of tracer 0 first.
 * chi       : [D] FP64 output.
 * vel       : [D][3] FP64 output, or NULL.
 * Errors: VOFMT_E_ARG (synchronises) if a label 1..K has no cells;
 *         VOFMT_E_EXTENT if a drop spans n/2 or more cells along an axis (the
 *         outputs are then still written).
 */
int vofmt_drop_shapes(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, const double *c,
                      const int32_t *labels, const int32_t *ndrops_host, const double *sx, const double *sy,
                      const double *sz, double *inertia, double *chi, double *vel, hipStream_t stream);

/*
 * Moments and shapes of every drop in one pass over the labels (the
 * combination of vofmt_drop_moments and vofmt_drop_shapes, each drop's cells
 * summed once): vol and xyz as vofmt_drop_moments gives them (the centroid
 * summed about the drop's box centre, so it may differ from that call's in
 * the last bits), inertia, chi and vel as vofmt_drop_shapes.
 * vol, xyz, inertia, chi: required outputs; vel with sx, sy, sz or all NULL.
 * Errors: as vofmt_drop_shapes.
 */
int vofmt_drop_moments_shapes(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, const double *c,
                              const int32_t *labels, const int32_t *ndrops_host, const double *sx, const double *sy,
                              const double *sz, double *vol, double *xyz, double *inertia, double *chi, double *vel,
                              hipStream_t stream);

/*
 * Reassign drops in near contact to other tracers (Steps 1-4 of section
 * "The no-coalescence.h algorithm"). Two distinct drops are neighbours when
 * an occupied cell of each lies at a periodic offset o with |o|^2 <
 * (1 + gap_cells)^2 (o = 0 included across tracers). Drops are visited in
 * ascending (tracer, label); a drop moves when an earlier neighbour has its
 * current tracer, to the smallest tracer not used by any of its neighbours,
 * or to a new tracer when all are used. Moved cells are cleared in the old
 * field and added to the new one; new tracer fields start from zero.
 *
 * ntracers_host: in/out host int32: number of tracers in use (synchronises).
 * max_tracers  : capacity of c; VOFMT_E_CAPACITY (nothing modified) if needed.
 * c            : [max_tracers][nz][ny][nx] FP64, in/out.
 * labels, ndrops_host: from vofmt_label_drops on the same c.
 * new_tracer   : [D] int32 device output: tracer of every drop afterwards.
 * nmoved_host  : host int32 output: number of drops moved.
 */
int vofmt_recolor_tracers(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t *ntracers_host,
                          int32_t max_tracers, double *c, const int32_t *labels, const int32_t *ndrops_host,
                          double gap_cells, int32_t *new_tracer, int32_t *nmoved_host, hipStream_t stream);

/*
 * The same reassignment with the near-contact criterion of Steps 1-3 read
 * literally (section "The no-coalescence.h algorithm", the near-contact
 * criterion figure), selectable beside the distance threshold above:
 *   - within a tracer, two drops are neighbours (a conflict) when a cell with
 *     no drop of that tracer (label 0: "C_i = 0" at the centre) has a cell of
 *     one drop and a cell of the other at opposite offsets +o, -o of the
 *     5x5x5 stencil, o in {-2..2}^3 \ {0} (Step 1, "C_i > 1" read as C_i > 0;
 *     Step 3, different tags);
 *   - across tracers, two drops are in contact (Step 4: the tracers a moved
 *     drop must avoid) when cells of the two lie within 4 cells of each other
 *     along every axis, the reach of the stencil, overlap included (a
 *     reading: the paper does not define this contact).
 * Visiting order, choice of the new tracer, cell moves, arguments, outputs,
 * scratch and errors as for vofmt_recolor_tracers (no gap argument). Extra
 * scratch: one 64-bit occupancy word per 64-cell row segment per tracer.
 */
int vofmt_recolor_tracers_stencil(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t *ntracers_host,
                                  int32_t max_tracers, double *c, const int32_t *labels, const int32_t *ndrops_host,
                                  int32_t *new_tracer, int32_t *nmoved_host, hipStream_t stream);

/*
 * Tracer compaction: the number of tracers in use, N(t), is what the paper
 * reports for its runs (section "The no-coalescence.h algorithm"); a tracer
 * holding no drop (every value at or below the labelling threshold) is
 * retired here, the other fields keep their order and move down over the
 * gaps, and the freed fields are set to zero.
 *
 * ntracers_host : in: N; out: the tracers kept.
 * c             : [N][nz][ny][nx] FP64, in place.
 * ndrops_host   : [N] drop counts (vofmt_label_drops); labels computed
 *                 before the call are invalid afterwards.
 * new_index_host: [N] host output, the new position of each tracer or -1.
 * discarded_host: host output, the sum of the retired fields' values (in a
 *                 fixed order, reproducible).
 * Synchronises the stream.
 */
int vofmt_compact_tracers(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t *ntracers_host, double *c,
                          const int32_t *ndrops_host, int32_t *new_index_host, double *discarded_host,
                          hipStream_t stream);

/*
 * Nearest-particle statistics (section "Nearest particle statistics").
 * For each drop i: the minimum-image vectors r_ij = x_j - x_i (per axis:
 * subtract L if r > L/2, add L if r <= -L/2), d2 = (rx^2 + ry^2) + rz^2, the
 * nearest set {j != i : d2 = min} (exact equality), N_i its size and the tie
 * weight h_ij = 1/N_i of eq. (4). Every nearest pair is binned (eqs. 8 and
 * 10): radial bin k with r2_edges[k] <= d2 < r2_edges[k+1]; polar bin m =
 * number of interior edges e = 1..ntheta-1 with cos(theta) <= cos_edges[e],
 * theta from the vertical axis, decided without sqrt as
 * rv*|rv| <= (ce*|ce|)*d2. Weights are integers in units of 1/720720; pairs
 * outside the radial range go to hist_fixed[nr*ntheta]. Moments (eqs. 11,
 * 14, as averages over the E = n events): M = (1/E) sum h r, R = (1/E) sum h r r^T,
 * and the deviatoric part A = R - (tr R / 3) delta of the second-moment
 * section (its "3 tr(R)" read as tr(R) = R : delta).
 *
 * xyz       : [n][3] FP64 drop centroids (cells). box: [3] HOST FP64.
 * r2_edges  : [nr+1] HOST FP64, ascending. cos_edges: [ntheta+1] HOST FP64, descending.
 * nn_index  : [n] int32 output (smallest nearest j). nn_ties: [n] int32 output (N_i).
 * hist_fixed: [nr*ntheta + 1] uint64 output. M: [3], R: [9] FP64 outputs.
 * A         : [9] FP64 output, or NULL.
 * Synchronises the stream (host staging of the edges). Scratch: 16 bytes per
 * drop and candidate slice (at most 64 slices) plus 104 bytes per drop.
 */
int vofmt_nearest_pair_stats(vofmt_ctx *ctx, int32_t n, const double *xyz, const double *box, int32_t vertical_axis,
                             int32_t nr, int32_t ntheta, const double *r2_edges, const double *cos_edges,
                             int32_t *nn_index, int32_t *nn_ties, uint64_t *hist_fixed, double *M, double *R,
                             double *A, hipStream_t stream);

/*
 * vofmt_nearest_pair_stats for callers that cannot allocate memory: code
 * under HIP graph capture, serving loops, harnesses that forbid allocation.
 * Same operation, arguments, outputs and results (bit for bit) as
 * vofmt_nearest_pair_stats, but no device or host memory is allocated and
 * the stream is not synchronised: the kernels work in a fixed array of the
 * library (4.8 MiB per device, held until the process ends) and the bin
 * edges travel as a kernel argument. Limits: n <= 8192 drops and
 * nr + ntheta + 2 <= 384 edges, else VOFMT_E_ARG (nothing enqueued). Every
 * call on one device shares that device's array: calls that overlap on a
 * device (any context or stream) race. VOFMT_E_HIP if the array's device
 * address could not be found when the context was created.
 */
int vofmt_nearest_pair_stats_noalloc(vofmt_ctx *ctx, int32_t n, const double *xyz, const double *box,
                                     int32_t vertical_axis, int32_t nr, int32_t ntheta, const double *r2_edges,
                                     const double *cos_edges, int32_t *nn_index, int32_t *nn_ties,
                                     uint64_t *hist_fixed, double *M, double *R, double *A, hipStream_t stream);

/*
 * Probability densities of the nearest-particle vector (section "Nearest
 * particle statistics", eqs. 8 and 10) from a histogram of
 * vofmt_nearest_pair_stats, or the sum of several over time (the paper
 * averages over all events E):
 *   P_nst(r, theta) = E_km / (E 2 pi r^2 sin(theta) dr dtheta),
 *   P_r-nst(r)      = sum_m E_km / (E 4 pi r^2 dr),
 * at the bin centres r = (r_k + r_k+1)/2, theta = (theta_m + theta_m+1)/2
 * (the paper writes the left edges, which makes the first radial and polar
 * bins singular). Operations in the written order, left to right.
 *
 * r_edges    : [nr+1] HOST FP64, ascending, r_edges[0] >= 0: the radii whose
 *              squares were the histogram's r2_edges.
 * theta_edges: [ntheta+1] HOST FP64, ascending within [0, pi]: the polar
 *              angles whose cosines were its cos_edges.
 * hist_fixed : [nr*ntheta] uint64 device, weights in units of 1/720720 (the
 *              overflow slot, if present, is not read).
 * events     : E, the number of drops summed over the histograms (>= 1).
 * P          : [nr][ntheta] FP64 device output. Pr: [nr] FP64 device output.
 * Synchronises the stream (host staging of the edges).
 */
int vofmt_pair_pdfs(vofmt_ctx *ctx, int32_t nr, int32_t ntheta, const double *r_edges, const double *theta_edges,
                    const uint64_t *hist_fixed, int64_t events, double *P, double *Pr, hipStream_t stream);

/*
 * Height-function curvature of one tracer field (the paper computes kappa_i
 * of every tracer "as for a single tracer", section "The no-coalescence.h
 * algorithm"; method: fixed 7-cell height columns). For each interface cell
 * (c more than 1e-12 inside (0, 1)) the Mixed-Youngs-Centred normal orders the column axes by
 * decreasing |m_d|; the first axis whose 3x3 columns all run from a full cell
 * (c >= 1-1e-6, on the phase side) to an empty one (c <= 1e-6) gives the
 * column sums H(u,v) over offsets -3..3 and
 *   kappa*Delta = -[Hxx(1+Hy^2) + Hyy(1+Hx^2) - 2 Hxy Hx Hy] / (1+Hx^2+Hy^2)^{3/2}
 * (+2/R on a sphere of radius R cells; negative for a bubble).
 *
 * c     : [nz][ny][nx] FP64, one tracer.
 * kappa : [nz][ny][nx] FP64 output, kappa*Delta, NaN where undefined.
 * status: [nz][ny][nx] uint8 output: 0 not an interface cell, 1..3 valid on
 *         the 1st..3rd axis tried, 4 no valid axis.
 * The mixed cells are first gathered into a list (scratch: one int32 per
 * cell), then one thread per listed cell evaluates the columns.
 */
int vofmt_curvature_hf(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *c, double *kappa,
                       uint8_t *status, hipStream_t stream);

/*
 * Surface-tension force of all tracers on the cell faces: the sum over the
 * tracers of gamma kappa_i grad C_i (section "The no-coalescence.h
 * algorithm"), in the balanced-force face-centred form (Popinet 2018). On the
 * lower d-face of cell p, between m = p - e_d (periodic) and p:
 *   F_d[p] = gamma * sum_i phi_i (C_i[p] - C_i[m]),
 * phi_i = (kappa_i[p] + kappa_i[m]) / 2 where both are defined, the defined
 * one where only one is; no contribution where neither is or where C_i[p] ==
 * C_i[m]. Tracers are summed in increasing order, then scaled by gamma.
 *
 * c     : [ntracers][nz][ny][nx] FP64 volume fractions.
 * kappa : [ntracers][nz][ny][nx] FP64 curvature kappa*Delta (as written by
 *         vofmt_curvature_hf or vofmt_curvature_mlp), NaN where undefined.
 * gamma : surface-tension coefficient (finite).
 * fx, fy, fz: [nz][ny][nx] FP64 outputs on the lower x-, y- and z-faces, in
 *         units of gamma per cell width squared; with ntracers == 0 they are
 *         set to zero.
 * Streams every tracer's c and kappa once; no scratch memory.
 */
int vofmt_csf_force(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, int32_t ntracers, const double *c,
                    const double *kappa, double gamma, double *fx, double *fy, double *fz, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Learned curvature (not in the paper, which uses height functions): a
 * multilayer perceptron 27 (zero-padded to 32) -> 128 -> 128 -> 1 with ReLU,
 * mapping the canonical 3x3x3 stencil of a mixed cell to kappa*Delta.
 *
 * Parameters: one FP32 array of VOFMT_MLP_NPARAMS values,
 *   W1[32][128] (input k, unit j) | b1[128] | W2[128][128] | b2[128] |
 *   W3[128] | b3 | 3 floats of padding,
 * owned by the caller, device memory. Arithmetic: the matrix products run on
 * the BF16 matrix cores with FP32 accumulation; their weights are rounded to
 * BF16 (nearest even) for each use, the first-layer activations and the
 * upstream gradients are rounded to BF16, and each input x enters as two BF16
 * numbers hi = bf16(x), lo = bf16(x - hi) times the same weights. The biases
 * are FP32 and enter the forward products' FP32 accumulation: b1 as three
 * BF16 numbers whose sum is b1 (exact for |b1| above 2^-100), b2 as the
 * initial accumulator. The last layer is an FP32 dot product of the unrounded
 * second-layer activations with the FP32 W3. Loss and Adam in FP32. Every
 * batch reduction is done in a fixed order, so results are reproducible bit
 * for bit on a given device (the batch's 64-sample tiles are split into at
 * most one contiguous range per compute unit).
 * ------------------------------------------------------------------------ */
#define VOFMT_MLP_NPARAMS 20868

/*
 * Forward pass on m stencils.
 * x    : [m][27] FP32 canonical stencils, order (ax+1) + 3(ay+1) + 9(az+1).
 * y    : [m] FP32 output, kappa*Delta of the canonical stencil.
 * acts : nullable; [m] records of 768 bytes output: the first-layer
 *        activations h1 as BF16 [128] (bytes 0..255) and the second-layer
 *        activations h2 as FP32 [128] (bytes 256..767).
 * Errors: VOFMT_E_ARG for m < 0 or null pointers (m = 0 is a no-op).
 */
int vofmt_mlp_forward(vofmt_ctx *ctx, const float *params, int32_t m, const float *x, float *y, uint8_t *acts,
                      hipStream_t stream);

/*
 * One training step on a batch of m stencils: forward, backward and one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8, 1-based step, learning rate lr) on
 * the FP32 masters params, adam_m, adam_v (all VOFMT_MLP_NPARAMS, updated in
 * place). Loss: mean over the batch of (y - t)^2 / max(|t|, 0.05)^2.
 * y_target : [m] FP32 target kappa*Delta of the canonical stencils.
 * grads    : nullable; [VOFMT_MLP_NPARAMS] FP32 output, the batch gradient.
 * trace    : nullable; [m] records of 1280 bytes output: the 768-byte
 *            activation record of vofmt_mlp_forward, then dL/dz2 and dL/dz1
 *            as BF16 [128] each, as rounded for the products.
 * loss_host: HOST output, the batch loss before the update (synchronises).
 * Errors: VOFMT_E_ARG for m < 1, step < 1, lr < 0 or null pointers.
 */
int vofmt_mlp_train_step(vofmt_ctx *ctx, float *params, float *adam_m, float *adam_v, int32_t step, float lr,
                         int32_t m, const float *x, const float *y_target, float *grads, uint8_t *trace,
                         float *loss_host, hipStream_t stream);

/*
 * Canonical stencils of the interface cells (c more than 1e-12 inside (0, 1))
 * of one field, in
 * increasing linear cell order. Canonicalisation over the 48 symmetries of
 * the cube: reflect the axes along which the Mixed-Youngs-Centred normal is
 * negative, order the axes by increasing |m_d| (ties: lower axis first), and
 * when the centre exceeds 1/2 replace c by 1 - c (sign -1: the curvature
 * changes sign). Periodic neighbours.
 * c          : [nz][ny][nx] FP64, one tracer.
 * capacity   : length of the outputs; VOFMT_E_ARG if fewer than the mixed cells.
 * xs         : [capacity][27] FP32 output. cell: [capacity] int32 linear cell
 *              index. sign: [capacity] int8, +1 or -1.
 * count_host : HOST output, the number of mixed cells (synchronises).
 */
int vofmt_mlp_stencils(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *c, int32_t capacity,
                       float *xs, int32_t *cell, int8_t *sign, int32_t *count_host, hipStream_t stream);

/*
 * Curvature of one tracer by the network with height functions as the
 * fallback: for every interface cell (c more than 1e-12 inside (0, 1))
 * kappa = sign * MLP(canonical stencil); where
 * |kappa| < kappa_lo (radii the 3x3x3 stencil cannot resolve) or the
 * stencil holds two interfaces (on the canonicalised block, MYC's
 * centred-columns orientation along the axis of the largest |m_d| disagrees
 * with the height functions' orientation there, full end low when
 * m_d >= 0), the height function is evaluated and replaces it when valid.
 * status: 0 not a mixed
 * cell (kappa NaN); 8 the network's value; 1..3 the height function's value
 * (valid on the 1st..3rd axis tried); 12 the network's value where the
 * height function was tried and had no valid axis.
 * nmixed_host: nullable HOST output, the number of mixed cells (the call
 *              synchronises once to size its work).
 */
int vofmt_curvature_mlp(vofmt_ctx *ctx, int32_t nx, int32_t ny, int32_t nz, const double *c, const float *params,
                        double kappa_lo, double *kappa, uint8_t *status, int32_t *nmixed_host, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched advection: many boxes of uneven sizes and tracer counts, each
 * advanced exactly as vofmt_advect would (eq. 3 of the paper per tracer,
 * direction-split sweeps in the order (g, g+1, g+2) mod 3 of global step g),
 * in one graph launch. The results are bit-identical to one vofmt_advect
 * call per box with the same step0 and nsteps, for every tuning.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t nx, ny, nz;  /* box size in cells (x fastest) */
  int32_t ntracers;
  double *c;           /* [ntracers][nz][ny][nx] FP64, device, advanced in place */
  const double *sx, *sy, *sz; /* face Courant numbers, device, as for vofmt_advect */
} vofmt_box;

typedef struct {
  int32_t chunk;             /* cells per thread along the marching axis: 8, 16, 32 or 64 */
  int32_t workgroups_per_cu; /* persistent grid: workgroups per compute unit, 1..32 */
} vofmt_tuning;

/*
 * boxes  : HOST array of nboxes descriptors (device pointers inside). Boxes
 *          must not share fields.
 * tuning : HOST, nullable (chunk 32, 8 workgroups per CU).
 * The launch sequence of all sweeps is captured into a HIP graph on the
 * context's own stream and launched on `stream`; a call with the same boxes,
 * tuning, nsteps and step0 mod 3 relaunches the cached graph. A call that
 * builds a new graph synchronises `stream` once (table upload). Scratch: per
 * box a second field copy, a face-flux array, the c > 0.5 bits and the lists
 * of mixed cells, in one slab owned by the context.
 * Errors: VOFMT_E_ARG for bad sizes, null pointers, ntracers*cells >= 2^32 or
 * a bad tuning; VOFMT_E_HIP / VOFMT_E_NOMEM from the runtime.
 */
int vofmt_advect_batched(vofmt_ctx *ctx, int32_t nboxes, const vofmt_box *boxes, int64_t step0, int32_t nsteps,
                         const vofmt_tuning *tuning, hipStream_t stream);

/*
 * Autotuner of vofmt_advect_batched: advances copies of the boxes' fields
 * (the caller's data is untouched) with each candidate tuning -- chunk
 * {16, 32, 64} x workgroups per CU {2, 4, 8, 16} -- for nsteps steps, times
 * each graph launch with HIP events (best of two), and returns the fastest.
 * best_host: HOST output. best_ms_host: nullable HOST output, its time.
 * Synchronises. Scratch: one copy of every field.
 */
int vofmt_autotune_batched(vofmt_ctx *ctx, int32_t nboxes, const vofmt_box *boxes, int32_t nsteps,
                           vofmt_tuning *best_host, float *best_ms_host, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Instrumentation: per-launch timing of this context's kernels with HIP
 * events recorded on the launch stream around every launch of the plain
 * advection passes, the curvature kernels and the network kernels (not inside
 * the batched graph). For benchmarks and tests; adds two event records per
 * launch while on.
 * ------------------------------------------------------------------------ */
/* Clears the records and starts recording. */
int vofmt_profile_start(vofmt_ctx *ctx);
/*
 * Stops recording and reports, per kernel kind in order of first launch:
 * names [max_kinds][48] (NUL-terminated), launches [max_kinds], total_ms
 * [max_kinds] (HOST arrays). nkinds_host gets the number of kinds seen (kinds
 * beyond max_kinds are not reported). Synchronises with every recorded event.
 */
int vofmt_profile_stop(vofmt_ctx *ctx, int32_t max_kinds, char *names, int32_t *launches, double *total_ms,
                       int32_t *nkinds_host);

#ifdef __cplusplus
}
#endif

#endif /* VOFMT_H */
