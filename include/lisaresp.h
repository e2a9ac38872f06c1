/*
 * lisaresp.h -- C ABI of the MI355X (gfx950) generic LISA time-domain
 * response: projection of the GW polarisations onto the six constellation
 * links, then first/second-generation Michelson TDI (arXiv:2204.06633,
 * Sec. IV).  FP64 throughout.
 *
 * Memory.  Every array argument is a DEVICE pointer owned by the caller
 * unless marked [host].  The library allocates, frees and synchronises
 * nothing in the compute calls (lr_orbits_init alone synchronises the stream
 * once, after its host-to-device copy), so the compute calls may be recorded
 * into a HIP graph.  Outputs must not overlap inputs.
 *
 * Streams.  `stream` is a hipStream_t passed as void*; NULL is the null
 * stream.  Work is enqueued in stream order; calls return as soon as it is
 * enqueued.
 *
 * Errors.  Argument checks happen on the host before any launch.  Every
 * call returns an lr_status; on failure lr_last_error() holds a message
 * (thread-local, valid until the next failing call on the thread).  A HIP
 * launch failure maps to LR_E_HIP with the runtime's text.
 *
 * Conventions (Sec. IV and Fig. 1).  Spacecraft 1..3, clockwise seen from
 * +z.  Link l = 0..5 is (receiver, emitter) = 12, 23, 31, 13, 32, 21, and
 * every per-link array is link-major: y[l * n + j].  Times are seconds,
 * positions metres in the SSB ecliptic frame.  A uniformly sampled series
 * s[j] sits at absolute time t0 + j * dt.
 *
 * Interpolation (Sec. IV.E).  Centred Lagrange interpolation of odd order
 * 1..31 (order + 1 taps): a value at fractional index j0 + eps, eps in
 * [0, 1), reads samples j0 - (order-1)/2 ... j0 + (order+1)/2.  Retarded
 * positions are formed as an integer sample index minus (delay / dt), with
 * the integer and fractional parts kept apart, so absolute times never limit
 * the FP64 precision.  Stencils never leave the caller's arrays: calls whose
 * padding is too small return LR_E_RANGE (see lr_projection_padding,
 * lr_tdi_padding).
 */
#ifndef LISARESP_H
#define LISARESP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LR_OK = 0,
    LR_E_ARG = 1,          /* null/aliased pointer, bad size, non-finite scalar */
    LR_E_RANGE = 2,        /* a stencil or an orbit evaluation leaves its data */
    LR_E_UNSUPPORTED = 3,  /* even or out-of-range order, unknown generation */
    LR_E_WORKSPACE = 4,    /* storage or workspace smaller than required */
    LR_E_HIP = 5           /* the HIP runtime reported an error */
} lr_status;

/* TDI output channels: X,Y,Z; A,E,T; or X,Y,Z followed by A,E,T. */
enum { LR_XYZ = 0, LR_AET = 1, LR_XYZ_AET = 2 };

/* Text of a status code; never NULL. */
const char *lr_status_str(int status);
/* Message of the last failing call on this thread ("" if none). */
const char *lr_last_error(void);
/* ABI version of this header (bumped on incompatible changes); the library
 * returns the version it was built with. */
#define LR_ABI_VERSION 5
int lr_abi_version(void);
/* The build-time tuning switches the library was compiled with, as
 * "NAME=value;NAME=value;..." (register budgets, load pipelining, the TDI
 * adjoint's fold): the product build has the kernel headers' defaults, a
 * variant build for measurements reports its own.  Static string; never
 * NULL. */
const char *lr_build_config(void);

/* ------------------------------------------------------------------------
 * Orbits.  The paper interpolates the orbit data once per run and keeps it
 * for every evaluation (Sec. IV.E).  Here the 9 position series (x, y, z of
 * spacecraft 1..3) and the 6 light travel times (link order above, at
 * reception time) are fitted with not-a-knot cubic splines on their coarse
 * uniform grid; kernels evaluate them at every sample time they need.
 * ---------------------------------------------------------------------- */
typedef struct {
    double t0;           /* absolute time of coarse sample 0 (s) */
    double dt;           /* coarse spacing (s), > 0 */
    int64_t n;           /* coarse samples, >= 4 */
    const void *coef;    /* device storage written by lr_orbits_init */
    double L_min, L_max; /* rigorous bounds of the light-time splines (s) */
    double R_max;        /* rigorous bound of |x| over the position splines (m) */
} lr_orbits;

/* Bytes of device storage lr_orbits_init needs for n coarse samples. */
size_t lr_orbits_bytes(int64_t n);

/* Fit the splines on the host and copy the coefficients to d_storage (the
 * caller keeps it alive while `out` is used).  x_sc [host][n][3][3] metres,
 * ltt [host][n][6] seconds.  Synchronises `stream` once.  Errors: LR_E_ARG
 * (n < 4, dt <= 0, non-finite data), LR_E_WORKSPACE (bytes too small),
 * LR_E_HIP. */
int lr_orbits_init(double t0, double dt, int64_t n, const double *x_sc, const double *ltt,
                   void *d_storage, size_t bytes, lr_orbits *out, void *stream);

/* [host only] The same spline fit without a device: fills `out` with t0, dt,
 * n and the bounds L_min, L_max, R_max (coef = NULL), which is all that
 * lr_projection_padding and lr_tdi_padding read -- so a caller can size its
 * padded buffers before anything is allocated or uploaded.  The handle is
 * not valid for the compute calls.  Errors: LR_E_ARG as lr_orbits_init. */
int lr_orbits_bounds(double t0, double dt, int64_t n, const double *x_sc, const double *ltt,
                     lr_orbits *out);

/* Samples of h+/hx that lr_project_links needs before the first and after
 * the last link sample it writes, for any sky position (from the orbit
 * bounds and the stencil half-width).  `orb` from lr_orbits_init or
 * lr_orbits_bounds. */
int lr_projection_padding(const lr_orbits *orb, int order, double dt, int64_t *front,
                          int64_t *back);

/* Samples of y that lr_tdi_combine needs before the first and after the last
 * output sample, for generation 1 (chains of <= 3 links) or 2 (<= 7). */
int lr_tdi_padding(const lr_orbits *orb, int order, int generation, double dt, int64_t *front,
                   int64_t *back);

/* ------------------------------------------------------------------------
 * Projection, Sec. IV.B, eq. (instrument response):
 *   y_ij(t) = [H_ij(t - L_ij(t) - k.x_j(t)/c) - H_ij(t - k.x_i(t)/c)]
 *             / (2 (1 - k.n_ij(t))),
 *   H_ij = h+ xi+(u, v, n_ij) + hx xix(u, v, n_ij),
 *   xi+ = (u.n)^2 - (v.n)^2,  xix = 2 (u.n)(v.n),
 * with k = -e_r, u = -e_phi, v = -e_theta of the ecliptic sky position
 * (lam, beta) (Sec. IV.A), n_ij = (x_i - x_j)/|x_i - x_j| and all orbit
 * quantities at the reception time t.
 *
 * hp, hc: [n_h] at t0_h + j*dt.  sky: device [2] = (lam, beta) in radians
 * (device-resident so that a captured graph can be replayed with new
 * angles).  Writes y[l * n_y + i] for the link sample at h-index
 * y_start + i, i = 0..n_y-1.  Requires y_start - front >= 0 and
 * y_start + n_y - 1 + back <= n_h - 1 (lr_projection_padding, valid for any
 * sky position), and the orbit grid to cover the link sample times.
 * n_y = 0 is a no-op.  Non-finite angles give non-finite y, never an
 * out-of-bounds access.
 * ---------------------------------------------------------------------- */
int lr_project_links(const lr_orbits *orb, double t0_h, double dt, int64_t n_h,
                     const double *hp, const double *hc, const double *sky, int order,
                     int64_t y_start, int64_t n_y, double *y, void *stream);

/* ------------------------------------------------------------------------
 * TDI, Sec. IV.C, eqs. (tdi1), (tdi2): Michelson X1 / X2 as signed sums of
 * link series delayed by chained delays D_{i1..in} x(t) = x(t - sum_k
 * L_{ik ik+1}(t)) (sums, all light times at the output time t); Y and Z by
 * the cyclic relabelling 1->2->3->1; optionally A = (Z-X)/sqrt2,
 * E = (X-2Y+Z)/sqrt6, T = (X+Y+Z)/sqrt3.
 *
 * y: [6][n_y] at t0_y + j*dt.  Writes out[c * n_out + i] for the sample
 * at y-index out_start + i, c = X,Y,Z (LR_XYZ), A,E,T (LR_AET) or
 * X,Y,Z,A,E,T (LR_XYZ_AET, out holds 6 rows).  Requires
 * out_start - front >= 0 and out_start + n_out - 1 + back <= n_y - 1
 * (lr_tdi_padding) and the orbit grid to cover the output times.
 * ---------------------------------------------------------------------- */
int lr_tdi_combine(const lr_orbits *orb, double t0_y, double dt, int64_t n_y, const double *y,
                   int generation, int order, int channels, int64_t out_start, int64_t n_out,
                   double *out, void *stream);

/* ------------------------------------------------------------------------
 * Adjoints.  Not in the paper; they are the exact transposes of the linear
 * maps above (derived from Sec. IV.B-IV.C and the interpolation of
 * Sec. IV.E), so that a likelihood gradient can flow from the TDI channels
 * back to h+, hx and the sky angles.  Each wave of 128 sources sums its
 * scatters in a register carry in a fixed order, the waves of a tile are
 * summed in a fixed order, and every output element receives at most two
 * tile sums (added onto zero, which commutes): results are bitwise
 * reproducible.  Exception: when dt is so small against the light times that
 * a wave's footprint does not fit LDS (about dt < L/50), LDS and global
 * atomics take over and results are reproducible to rounding only.
 * ---------------------------------------------------------------------- */

/* g_y = T^T g_out: transpose of lr_tdi_combine with the same arguments.
 * g_out: [3 or 6][n_out] laid out like `out`; g_y: [6][n_y], overwritten
 * (entries no output depends on are zero). */
int lr_tdi_adjoint(const lr_orbits *orb, double t0_y, double dt, int64_t n_y, int generation,
                   int order, int channels, int64_t out_start, int64_t n_out,
                   const double *g_out, double *g_y, void *stream);

/* Bytes of device workspace lr_project_adjoint needs for the sky gradient. */
size_t lr_project_adjoint_workspace(int64_t n_y);

/* (g_hp, g_hc) = P^T g_y: transpose of lr_project_links with respect to h+
 * and hx (same arguments), both [n_h] and overwritten.  If g_sky is not
 * NULL it receives d<g_y, y>/d(lam, beta) (device [2]); that needs hp, hc
 * and a device workspace of lr_project_adjoint_workspace(n_y) bytes (its
 * partial sums are reduced in a fixed order).  hp and hc may be NULL when
 * g_sky is NULL. */
int lr_project_adjoint(const lr_orbits *orb, double t0_h, double dt, int64_t n_h,
                       const double *hp, const double *hc, const double *sky, int order,
                       int64_t y_start, int64_t n_y, const double *g_y, double *g_hp,
                       double *g_hc, double *g_sky, void *work, size_t work_bytes,
                       void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as lr_project_adjoint, with the sky-gradient partial sums kept in a static
 * device array of lr_noalloc_scratch_bytes() bytes (1 MiB; one copy per GPU,
 * held until the process ends) instead of a caller workspace.  The library
 * allocates nothing.  With g_sky != NULL, n_y may be at most 16,777,216 link
 * samples (65,536 tiles of 256); larger n_y returns LR_E_WORKSPACE before
 * any launch.  Every call on one GPU shares that GPU's array, so calls that
 * overlap in time on one GPU (different streams, host threads) race; each
 * call overwrites all the partial sums it reads.  The first call on a device
 * looks up the array's device address (hipGetSymbolAddress). */
size_t lr_noalloc_scratch_bytes(void);
int lr_project_adjoint_noalloc(const lr_orbits *orb, double t0_h, double dt, int64_t n_h,
                               const double *hp, const double *hc, const double *sky, int order,
                               int64_t y_start, int64_t n_y, const double *g_y, double *g_hp,
                               double *g_hc, double *g_sky, void *stream);

/* ------------------------------------------------------------------------
 * White-noise likelihood, Sec. II.A eq. (like) with the channel sum of
 * Sec. IV.C, for noise of standard deviation sigma per sample and channel:
 *   loglike = -1/2 sum_k (data_k - h_k)^2 / sigma^2,
 *   g_h_k   = d loglike / d h_k = (data_k - h_k) / sigma^2.
 * h, data, g_h: device [n] (any channel-major layout, e.g. [3][n_out]);
 * loglike: device [1]; g_h may be NULL.  The sum runs over a fixed grid in a
 * fixed order (deterministic).  work: lr_loglike_workspace() bytes.
 * ---------------------------------------------------------------------- */
size_t lr_loglike_workspace(void);
int lr_loglike(const double *h, const double *data, int64_t n, double sigma, double *loglike,
               double *g_h, void *work, size_t work_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batches: many templates (sources, or MCMC walkers of one source; the
 * paper's sampler runs 4 temperatures x 50 walkers, Sec. II.B) whose outputs
 * share one time grid t0 + i*dt, evaluated by one persistent fused kernel:
 * projection and TDI in one pass with the link series kept on chip, and the
 * TDI interpolation coefficients (which depend on the orbits only) shared by
 * `group` templates at a time.  Durations may differ between templates.
 * Projection and TDI may use different orbits (the paper's hybrid
 * templates, Sec. V).
 * ---------------------------------------------------------------------- */
typedef struct {
    int64_t h_offset;    /* index of the template's h[0] in the batch h+ / hx arrays */
    int64_t n_h;         /* its h samples */
    int64_t out_start;   /* its h-index of output sample 0 (time t0) */
    int64_t n_out;       /* its output samples (>= 0) */
    int64_t out_offset;  /* index of its output block in the batch output array; the block
                            is rows x n_out, channel-major (rows 3, or 6 for LR_XYZ_AET) */
} lr_template;

/* Filled by lr_batch_prepare; treat as opaque.  Holds copies of the orbit
 * handles and offsets into the caller's device workspace. */
typedef struct {
    lr_orbits proj, tdi;
    double t0, dt;
    int order, generation, channels, group;
    int front, tile_out, blocks, adjoint;
    int tile, segment;   /* link samples per forward tile; tiles per forward work item */
    int64_t n_templates, n_items, n_tdi_items, n_proj_items, n_like_items;
    int64_t n_tdi_citems, n_padj_citems;
    int64_t gy_doubles, h_extent, out_extent;
    void *ws;
    size_t off[24];      /* workspace region offsets (bytes) */
} lr_batch;

/* Device workspace bytes for a batch.  With adjoint != 0 it includes the
 * link-gradient scratch of lr_response_adjoint (6 values per link sample of
 * every template). */
size_t lr_batch_workspace(const lr_template *t, int64_t n, const lr_orbits *tdi, double dt,
                          int order, int generation, int channels, int group, int tile,
                          int segment, int adjoint);

/* Validate a batch (per-template padding from lr_projection_padding /
 * lr_tdi_padding, orbit coverage, output blocks), build the work lists and
 * copy them into ws (synchronises `stream` once; call it outside graph
 * capture).  t: [host][n]; group = templates per work item (1, 2 or 4);
 * tile = link samples per forward tile (256, 512 or 1024, not 1024 with
 * group 4; 0 = 512): the autotuner's tile-length knob; segment = tiles per
 * forward work item (1..64; 0 = automatic): consecutive tiles of a work item
 * pass the TDI halo on in LDS, so that only the first computes the halo's
 * link samples (taken as 1 where the halo exceeds what the kernel carries;
 * lr_batch.segment holds the value used).  Results do not depend on group,
 * tile, segment or grid.  t0: absolute time of output sample 0.
 * Errors: LR_E_ARG, LR_E_RANGE, LR_E_UNSUPPORTED (dt so small that the TDI
 * stencil does not fit a tile, or an uncompiled group/tile pair),
 * LR_E_WORKSPACE, LR_E_HIP. */
int lr_batch_prepare(const lr_template *t, int64_t n, const lr_orbits *proj,
                     const lr_orbits *tdi, double t0, double dt, int order, int generation,
                     int channels, int group, int tile, int segment, int adjoint, void *ws,
                     size_t ws_bytes, lr_batch *out, void *stream);

/* Forward response of every template (Sec. IV.B-IV.C): hp, hc hold the
 * templates' h arrays at their offsets, sky is device [n][2] (lam, beta),
 * out receives each template's block (other elements untouched).  All
 * pointers are device memory owned by the caller.  Graph-capturable.  Calls
 * that share one lr_batch (its workspace holds the work counter) must not
 * overlap in time.  Errors: LR_E_ARG (unprepared batch, null pointer),
 * LR_E_HIP (launch). */
int lr_response(const lr_batch *b, const double *hp, const double *hc, const double *sky,
                double *out, void *stream);

/* lr_response with h+ and hx synthesised inside the fused kernel (each work
 * item writes the Galactic-binary waveform of Sec. III straight into its LDS
 * window) from parameter rows instead of read from HBM: params device [n][8]
 * = (A, f0, fdot, phi0, iota, psi, lam, beta) in the caller's order, sky
 * angles included.  Template k's h sample j (j in [0, n_h)) is the waveform
 * at t = (j - out_start) dt: waveform time 0 at output sample 0, the
 * convention of lr_gb_polarizations with k0 = -out_start.  Bit for bit equal
 * to lr_gb_polarizations followed by lr_response.  The templates' h_offset is
 * not used; the batch needs no h arrays.  Graph-capturable.  Compiled for
 * batches prepared with group 1 or 2 at tile 512 and group 2 at tile 1024
 * (the waveform code is its own kernel variant).  Errors: LR_E_ARG,
 * LR_E_UNSUPPORTED (another group/tile pair), LR_E_HIP. */
int lr_response_gb(const lr_batch *b, const double *params, double *out, void *stream);

/* Transpose of lr_response (needs a batch prepared with adjoint != 0):
 * g_out laid out like out; g_hp, g_hc like hp, hc over [0, h_extent),
 * overwritten; g_sky device [n][2] (d/d lam, d/d beta) or NULL (then hp, hc
 * may be NULL too).  Graph-capturable; calls sharing one lr_batch must not
 * overlap.  Results are bitwise reproducible unless dt is so small (below
 * about a fiftieth of the light time) that the scatter footprints do not fit
 * LDS; then atomics reorder the sums and results are reproducible to
 * rounding.
 * Errors: LR_E_WORKSPACE (batch prepared without adjoint), LR_E_ARG,
 * LR_E_HIP. */
int lr_response_adjoint(const lr_batch *b, const double *hp, const double *hc,
                        const double *sky, const double *g_out, double *g_hp, double *g_hc,
                        double *g_sky, void *stream);

/* Transpose of lr_response_gb down to the source parameters: g_params
 * device [n][8] receives d<g_out, out>/d(A, f0, fdot, phi0, iota, psi, lam,
 * beta) for every template (zeros for an empty one), g_out laid out like
 * out.  The TDI and projection adjoints run as in lr_response_adjoint, but
 * each projection tile turns its share of the h+/hx gradient straight into
 * the seven parameter-gradient sums of the waveform (Sec. III) and the sky
 * tiles synthesise h from the parameters, so no h or h-gradient arrays
 * exist; per-template sums are reduced in tile order (deterministic).
 * Needs a batch prepared with adjoint != 0.  Graph-capturable.  Errors:
 * LR_E_WORKSPACE (no adjoint workspace), LR_E_ARG, LR_E_UNSUPPORTED (dt so
 * small, below about L/50, that the projection footprints do not fit LDS),
 * LR_E_HIP. */
int lr_response_adjoint_gb(const lr_batch *b, const double *params, const double *g_out,
                           double *g_params, void *stream);

/* Per-template white-noise log-likelihood (as lr_loglike, Sec. II.A) of a
 * batch output: data laid out like out; loglike device [n] (0 for an empty
 * template); g_out (like out, or NULL) receives (data - out)/sigma^2 over
 * each template's block.  Deterministic fixed-order sums.  Graph-capturable;
 * calls sharing one lr_batch must not overlap.  Errors: LR_E_ARG (sigma <= 0
 * or not finite, null pointer), LR_E_HIP. */
int lr_batch_loglike(const lr_batch *b, const double *out, const double *data, double sigma,
                     double *loglike, double *g_out, void *stream);

/* Work-group count of lr_response's persistent launch (the autotuner's grid
 * knob).  lr_batch_prepare sets it to min(work items, CUs x resident groups
 * per CU); any value >= 1 is valid, groups beyond the resident ones start
 * late and find the work list drained.  Errors: LR_E_ARG. */
int lr_batch_set_grid(lr_batch *b, int blocks);

/* ------------------------------------------------------------------------
 * Frequency-domain likelihood, Sec. II.A (the noise-weighted inner product,
 * log L = -<d-h|d-h>/2, optimal SNR sqrt(<h|h>), extraction SNR
 * <d|h>/sqrt(<h|h>)), discretised as
 *   <a|b> = sum_{k=0}^{N/2} w_k Re(conj(a~_k) b~_k),
 *   a~_k  = dt sum_{j<N} a_j exp(-2 pi i k j / N),
 * every series zero-padded to N = lr_fd_length(n) samples; w_k = 4 df /
 * S_n(f_k) with df = 1/(N dt) is supplied by the caller (0 drops a bin).
 * Channels: A, E (sharing the weights w_ae) and optionally T (weights w_t),
 * each a series of n samples.  For every template h and the data d:
 *   stats = (rr, hh, dh) = (<d-h|d-h>, <h|h>, <d|h>), summed over channels,
 *   g_h_j = d log L / d h_j = dt sum_{k=0}^{N/2} w_k Re(r~_k exp(+2 pi i k j / N)),
 * r = d - h.  The transforms run in FP64 on power-of-two sizes; results
 * match an exact evaluation to FFT rounding (relative ~1e-15 log2 N of the
 * weighted norms).
 * ---------------------------------------------------------------------- */

/* Filled by lr_fd_prepare; treat as opaque. */
typedef struct {
    int64_t n, n_fft, max_batch;
    int channels, log2n, passes, q[3];
    double dt;
    void *ws;
    size_t ws_bytes;
    size_t off[6];       /* workspace region offsets (bytes) */
} lr_fd_plan;

/* Transform length for n samples: the smallest power of two >= max(n, 4096);
 * -1 if n < 1 or n > 2^24. */
int64_t lr_fd_length(int64_t n);

/* Device workspace bytes of a plan for n samples, channels 2 (A, E) or 3
 * (A, E, T), and up to max_batch templates per launch sequence; 0 if the
 * arguments are invalid.  About (48 + 32 channels/2 x max_batch) bytes per
 * transform point. */
size_t lr_fd_workspace(int64_t n, int channels, int64_t max_batch);

/* Build a plan in the caller's workspace ws (device, ws_bytes >=
 * lr_fd_workspace): twiddle tables, the weights in transform order and the
 * data spectrum.  data: device, channel c's n samples at data + c *
 * data_cstride (data_cstride >= n); w_ae, w_t: device [N/2 + 1] (w_t
 * unused, may be NULL, when channels == 2).  The inputs are read on
 * `stream` and may be freed once it has passed this call; the plan keeps
 * pointers into ws only.  Errors: LR_E_ARG (sizes, null pointers, overlap
 * with ws), LR_E_UNSUPPORTED (n > 2^24), LR_E_WORKSPACE, LR_E_HIP. */
int lr_fd_prepare(int64_t n, int channels, double dt, const double *data, int64_t data_cstride,
                  const double *w_ae, const double *w_t, int64_t max_batch, void *ws,
                  size_t ws_bytes, lr_fd_plan *out, void *stream);

/* Statistics (and gradient) of n_templates templates: template t's channel c
 * at h + t * t_stride + c * c_stride (c_stride >= n, t_stride >= (channels -
 * 1) * c_stride + n); stats: device [n_templates][3] (rr, hh, dh); g_h: NULL
 * or device, laid out like h, receives d log L / d h (every sample of every
 * channel overwritten).  Templates are processed max_batch at a time.
 * Deterministic (fixed-order sums).  Graph-capturable; calls sharing one plan
 * (its workspace) must not overlap.  Errors: LR_E_ARG (unprepared plan, null
 * pointer, strides, g_h or stats overlapping an input or the workspace),
 * LR_E_HIP. */
int lr_fd_loglike(const lr_fd_plan *p, int64_t n_templates, const double *h, int64_t t_stride,
                  int64_t c_stride, double *stats, double *g_h, void *stream);

/* ------------------------------------------------------------------------
 * Galactic-binary polarisations, Sec. III, for n templates on one time grid:
 *   Phi(t) = 2 pi (f0 t + fdot t^2/2 + fddot t^3/6) + phi0,
 *   fddot = 11 fdot^2 / (3 f0),
 *   a+ = -(1 + cos^2 iota) A cos Phi,   ax = -2 cos(iota) A sin Phi,
 *   h+ = cos(2 psi) a+ - sin(2 psi) ax, hx = sin(2 psi) a+ + cos(2 psi) ax,
 * at t_j = (k0 + j) dt, j = 0 .. n_h - 1 (t = 0 at the template's first
 * output sample: k0 = -out_start).  The phase is evaluated in cycles with
 * the product f0 t split exactly and whole cycles removed, so its rounding
 * stays ~1e-15 rad over years.  params: device [n][8] = (A, f0, fdot,
 * phi0, iota, psi, lambda, beta) (lambda, beta unused here); f0 <= 0 gives
 * non-finite output, not an error (the values are not read on the host).
 * ---------------------------------------------------------------------- */

/* hp, hc: device, template t's samples at hp + t * h_stride (h_stride >=
 * n_h), overwritten.  Graph-capturable.  Errors: LR_E_ARG (sizes, dt,
 * overlap), LR_E_UNSUPPORTED (n > 65535), LR_E_HIP. */
int lr_gb_polarizations(const double *params, int64_t n, int64_t k0, int64_t n_h, double dt,
                        double *hp, double *hc, int64_t h_stride, void *stream);

/* Device workspace bytes of lr_gb_polarizations_adjoint. */
size_t lr_gb_adjoint_workspace(int64_t n, int64_t n_h);

/* g_params[t][k] = sum_j (g_hp[t][j] dh+/dparam_k + g_hc[t][j] dhx/dparam_k)
 * (the transpose of the linearised lr_gb_polarizations; fddot's dependence
 * on f0 and fdot included; the lambda and beta entries are 0).  g_hp, g_hc
 * laid out like hp, hc; g_params device [n][8], overwritten.  Sums are
 * per-block partials reduced in a fixed order (deterministic).
 * Graph-capturable.  Errors: LR_E_ARG, LR_E_UNSUPPORTED, LR_E_WORKSPACE,
 * LR_E_HIP. */
int lr_gb_polarizations_adjoint(const double *params, int64_t n, int64_t k0, int64_t n_h,
                                double dt, const double *g_hp, const double *g_hc,
                                int64_t h_stride, double *g_params, void *work,
                                size_t work_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LISARESP_H */
