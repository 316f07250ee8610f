/*
 * af.h -- C ABI of the MI355X (gfx950) lens-aware differentiable beamformer.
 *
 * The library evaluates, at every optimiser step, the hot path of lens-aware
 * ultrasound autofocusing (Frey et al., "Lens-Aware Differentiable Beamforming
 * for In Vivo Distributed Aberration Correction with Curvilinear Transducers"):
 *   bent-ray travel times (Fermat refraction through the lens, Eqs. 7-8, then
 *   the bicubic path integral of slowness, Eq. 1 and Section III-A), complex-IQ
 *   delay-and-sum over transmit x receive x point with phase rotation (Eq. 5),
 *   the common-midpoint phase-error loss with deadzone regularisers (Eqs. 10-12)
 *   and, by hand-written adjoints, its gradient with respect to the slowness grid.
 *
 * Conventions
 *   Units: mm, microseconds, MHz; speed in mm/us, slowness in us/mm.
 *   Coordinates: x lateral, z into the body; the origin is the centre of
 *   curvature of a curvilinear array (any point of the element line for a
 *   linear array).  Host arrays are read during the call and never retained; device
 *   pointers are caller-owned and must stay valid until the work enqueued on
 *   the context's stream has finished.  Every call that takes device pointers
 *   only enqueues work on that stream (no host synchronisation); results are
 *   visible after the caller synchronises the stream.
 *   Complex data are interleaved float pairs (re, im).
 *   Errors: every call returns an af_status; nothing throws across the ABI.
 *   af_last_error() gives a human-readable reason for the last failure.
 *   A context is not thread-safe; use one per host thread / stream.
 */
#ifndef AF_H_
#define AF_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct af_ctx af_ctx;

typedef enum {
  AF_OK = 0,
  AF_ERR_ARG = -1,      /* invalid argument (sizes, geometry, coverage) */
  AF_ERR_STATE = -2,    /* call out of order (e.g. beamform before set_slowness) */
  AF_ERR_HIP = -3,      /* HIP runtime error; see af_last_error */
  AF_ERR_OOM = -4,      /* device allocation failed */
  AF_ERR_NUMERIC = -5   /* slowness not finite and positive (af_set_slowness, af_simulate) */
} af_status;

typedef struct { float x, y; } af_complex;

/* Objective weights (Eq. 12 plus an optional speckle-brightness term).
 * total = L_CMPE + w1 R_TV + w2 R_SV - w_sb * SB / sb_ref. */
typedef struct {
  float w1, kx1, kz1;     /* first-order deadzone weight and thresholds (Eq. 10) */
  float w2, kx2, kz2;     /* second-order deadzone weight and thresholds (Eq. 11) */
  float rho_thresh;       /* correlation threshold of a valid CMPE pair */
  float w_sb, sb_ref;     /* speckle-brightness weight and reference (sb_ref > 0) */
} af_loss_params;

typedef struct { float lr, beta1, beta2, eps; } af_adam_params;

/* Layout of the terms vector written by forward / loss_and_grad / autofocus_step. */
enum {
  AF_TERM_CMPE = 0, AF_TERM_TV = 1, AF_TERM_SV = 2, AF_TERM_SB = 3,
  AF_TERM_TOTAL = 4, AF_TERM_NVALID = 5, AF_TERM_CMED = 6, AF_N_TERMS = 8
};

/* Create a context on HIP device `device`, enqueueing on `stream` (a hipStream_t;
 * NULL = the null stream).  Errors: AF_ERR_ARG (bad device), AF_ERR_HIP. */
af_status af_create(af_ctx** out, int device, void* stream);
/* Free every device buffer the context owns.  Safe on NULL. */
void af_destroy(af_ctx* ctx);
/* Last error text of `ctx`; with ctx NULL, why this thread's last failed
 * af_create failed (a static text if none did); never NULL. */
const char* af_last_error(const af_ctx* ctx);

/* Static acquisition and imaging geometry (Section II-A, Eqs. 2-5; Section III-A).
 *   elem_xz   [n_elem][2] element centres (host, float64): on a circular arc
 *             centred at the origin, in increasing polar angle (curvilinear
 *             array, concentric lens); or on one line z = const, in increasing x
 *             (linear array, flat lens: taken when every z agrees to 1e-9 of the
 *             array's size).  Element orientation follows Eq. 3.
 *   pix_xz    [n_pix][2] patch centres (host, float64); each patch is a
 *             patch x patch kernel of points at patch_spacing (lambda/2), point m
 *             offset by ((m % patch - patch/2), (m / patch - patch/2)) * spacing.
 *   n_samples, fs, t0, fd: channel-data samples per record, sampling rate,
 *             time of sample 0 and demodulation frequency of Eq. 5.
 *   block     S, elements per block; subapertures span two blocks (stride S).
 *   fnum      F of the apodisation |x'| <= (F/2) z' (Eq. 4, literal form).
 *   n_seg     ray segments after the lens (N_segments).
 * Caller order of points: p = q * patch^2 + m for pixel q, patch point m.
 * Tiles whose CMPE staging (the subaperture images and pair entries of their
 * span of active blocks) does not fit LDS run that stage from device memory the
 * context owns, at some cost in speed; at 3 x 3 patches a span of 16 blocks fits
 * where it reaches an end of the array, whose pair range is shorter.
 * Errors: AF_ERR_ARG if n_elem < 3, block does not divide n_elem, patch is not
 * 1 or 3, sizes are not positive, the elements are out of order or the active
 * element set of a point is not contiguous; AF_ERR_OOM. */
af_status af_set_geometry(af_ctx* ctx, int n_elem, const double* elem_xz, int n_pix,
                    const double* pix_xz, int patch, double patch_spacing,
                    int n_samples, double fs, double t0, double fd, int block,
                    double fnum, int n_seg);

/* Lens model of the beamformer (Section II-B).  The physical lens is a layer of
 * thickness d_lens (elements sit that far behind the concentric lens arc, or
 * below the flat lens surface z_elem + d_lens of a linear array) and speed
 * c_lens; t_ttp is the time-to-peak offset of the received envelope, added to
 * every round trip.  `mode` selects how the beamformer accounts for the lens:
 *   AF_LENS_BENT          bent rays refracted at the lens surface by Fermat's
 *                         principle (Eqs. 7-8), the default;
 *   AF_LENS_CONVENTIONAL  straight rays from the elements plus the scalar lens
 *                         offset of Eq. 6, read as the round-trip excess time of
 *                         crossing the lens along the element normal at c_lens
 *                         instead of c_ref: 2 d_lens (1/c_lens - 1/c_ref);
 *   AF_LENS_NONE          straight rays from the elements and no lens term (the
 *                         uncorrected baseline of the paper's comparisons).
 * c_ref (mm/us) is used by AF_LENS_CONVENTIONAL only.  The channel-data
 * simulator (af_simulate) always uses the physical lens with bent rays.  With a
 * straight-ray mode the slowness grid must cover the element positions, where
 * the rays start (af_set_slowness checks it).
 * Errors: AF_ERR_ARG for d_lens < 0, c_lens <= 0, a non-finite t_ttp, an
 * unknown mode, or c_ref <= 0 with AF_LENS_CONVENTIONAL. */
enum { AF_LENS_BENT = 0, AF_LENS_CONVENTIONAL = 1, AF_LENS_NONE = 2 };
af_status af_set_lens(af_ctx* ctx, double d_lens, double c_lens, double t_ttp, int mode,
                      double c_ref);

/* Refraction-point rule of the lens model (Section III-A, model implementation):
 * n_search = 0 (the default) takes the exact Fermat stationary point (continuous
 * root, Eq. 8); n_search in [2, AF_MAX_SEARCH] takes the best of n_search lens
 * points evenly spaced in polar angle over the interval that holds the root:
 * from the element's polar angle to the crossing of the straight element-point
 * segment with the lens arc when c_lens <= c_med, else from that crossing to the
 * point's polar angle; least L1/c_lens + L2/c_med at the global mean speed wins
 * (the first on ties).  Applies to the table, the beamformer and the gradient
 * from the next call on; no effect with d_lens = 0.
 * Errors: AF_ERR_ARG for other values of n_search. */
#define AF_MAX_SEARCH 4096
af_status af_set_refraction_search(af_ctx* ctx, int n_search);

/* Reduction order of the gradient (the adjoint of Eq. 5 feeds every travel time
 * T[a][p] from the samples where element a transmits and from those where it
 * receives).  on = 0 (the default): the transmit-role sums, which span the work
 * items of several receive blocks, are added with floating-point atomics, so the
 * last bits of the gradient may differ between runs.  on = 1: every work item
 * writes its partial sums to a slab of its own (device memory the context owns:
 * per tile, active elements x receive blocks x 256 points, 4 bytes each) and the
 * path adjoint adds them in a fixed order, so loss and gradient are the same bit
 * for bit on every run, at a few percent more time.  Applies from the next call
 * on.  Errors: AF_ERR_ARG for other values, AF_ERR_OOM. */
af_status af_set_deterministic(af_ctx* ctx, int on);

/* Bounded-memory mode (recomputation instead of storage).  bytes = 0 (the
 * default): the travel-time table of every (element, point), its rays and the
 * block images of every point are held at once (for the clinical workload about
 * 2.3 GB, for the 192-element, 512 x 512 pixel one about 27 GB).  bytes > 0: the
 * points are processed in chunks of whole tiles whose table, rays, block images
 * and time gradient fit in about `bytes` of device memory (at least one tile per
 * chunk); af_loss_and_grad and af_autofocus_step then evaluate the loss over all
 * chunks first and, in the gradient pass, recompute each chunk's table and block
 * images instead of keeping them (about 1.5 times the work of the unbounded
 * call); af_beamform, af_travel_times and af_sweep run chunk by chunk.
 * af_forward, af_backward, af_channel_images and af_lag_one_coherence hand data
 * of every point across the boundary and return AF_ERR_STATE under a budget.
 * Takes effect at once (the chunk buffers are freed and sized again) or at
 * af_set_geometry.  Errors: AF_ERR_OOM, AF_ERR_HIP. */
af_status af_set_memory_budget(af_ctx* ctx, size_t bytes);

/* Slowness grid s ~ 1/c (Section III-A): node (i, j) at (x0 + j dx, z0 + i dz),
 * values [nz][nx] float32 at `s_dev` (device), copied on the context stream.
 * At most (nx+3)(nz+3) = 9600 padded nodes (e.g. 95 x 95).
 * The grid box must contain every evaluation point and the lens arc (the element
 * arc for a straight-ray lens model) over the angles of the elements and points
 * (AF_ERR_ARG otherwise); needs geometry and lens first (AF_ERR_STATE).
 * The copied values are read back and checked on the host, which synchronises
 * the stream: a node that is not finite and positive gives AF_ERR_NUMERIC, and
 * the context then has no slowness until the next successful call.
 * (af_autofocus_step reads its s_dev on the device only: a non-finite or
 * non-positive value there shows as total = NaN in its terms; the kernels then
 * treat the affected rays as masked, so no index leaves its buffer.) */
af_status af_set_slowness(af_ctx* ctx, int nx, int nz, double x0, double z0, double dx,
                    double dz, const float* s_dev);

/* Beamform at the current slowness (Eq. 5).  iq_dev: [n_elem][n_elem][n_samples]
 * demodulated FSA data (device), transmit-major.  Optional outputs (NULL = skip):
 *   blk_dev  [Nb][Nb][P] block-pair images B^blk[i][j](p), Nb = n_elem / block;
 *   img_dev  [P] full-aperture image (sum over all block pairs);
 *   maps_dev [3][n_pix] integrated CMPE (per-pixel mean phase error over valid
 *            pairs), coherence factor at the patch centres, and common-midpoint
 *            correlation coefficient (per-pixel mean rho over the pairs with
 *            energy, before the rho threshold) - global image-quality metrics
 *            of the Model Evaluation subsection.
 * Point order is the caller's (see af_set_geometry).  The CMPE map uses
 * rho_thresh from the most recent loss call (default 0.9).  The channel data
 * must be finite: samples of apodised-out element pairs are read and weighted
 * by zero, so a non-finite sample anywhere in a read window makes the result
 * non-finite. */
af_status af_beamform(af_ctx* ctx, const af_complex* iq_dev, af_complex* blk_dev,
                af_complex* img_dev, float* maps_dev);

/* Receive-channel images (Eq. 5 with the transmit aperture the whole array and
 * the receive aperture one element): x_dev[r][p] = sum_t h_t h_r
 * Psi_{t,r}(tau) exp(j 2 pi f_d tau), complex64 [n_elem][n_points] in caller
 * point order, device memory owned by the caller, at the current slowness.  The
 * focused per-channel signals of the coherence metrics of the Model Evaluation
 * subsection.  The library keeps an internal buffer of n_elem x points x 8 bytes
 * from the first call on.
 * Errors: AF_ERR_STATE before geometry, lens and slowness; AF_ERR_ARG for null
 * pointers; AF_ERR_OOM if the buffer cannot be allocated. */
af_status af_channel_images(af_ctx* ctx, const af_complex* iq_dev, af_complex* x_dev);

/* Lag-one coherence of every pixel (global image-quality metric of the Model
 * Evaluation subsection): over the pixel's patch points m and every pair of
 * adjacent receive elements (r, r+1) whose channel images both have energy
 * E = sum_m |x|^2 > 1e-30, the mean of Re(sum_m x_r conj(x_{r+1})) / sqrt(E_r
 * E_{r+1}); 0 if no pair qualifies.  loc_dev: float32 [n_pix] (device, caller
 * pixel order).  Same state, buffer and errors as af_channel_images. */
af_status af_lag_one_coherence(af_ctx* ctx, const af_complex* iq_dev, float* loc_dev);

/* Loss (Eq. 12, CMPE + regularisers - speckle term) and, if grad_dev != NULL,
 * its gradient dL/ds [nz][nx] (device, overwritten).  terms_dev: float[8]
 * (device), see AF_TERM_*.  Refraction points, c_med, apodisation and validity
 * masks are held constant in the gradient. */
af_status af_loss_and_grad(af_ctx* ctx, const af_complex* iq_dev, const af_loss_params* lp,
                     float* terms_dev, float* grad_dev);

/* Forward half of loss_and_grad for a split autograd: writes the terms and
 * gblk_dev [Nb][Nb][P_internal] (device, size from af_query(AF_Q_GBLK_ELEMS)),
 * the loss gradient with respect to the block images in the library's internal
 * point order.  No travel-time table outlives the call. */
af_status af_forward(af_ctx* ctx, const af_complex* iq_dev, const af_loss_params* lp,
               float* terms_dev, af_complex* gblk_dev);

/* Backward half: recomputes the travel-time table at the current slowness, runs
 * the DAS adjoint with gblk_dev (from af_forward at the same slowness) and the
 * path adjoint, adds the regulariser gradient, and writes grad_dev [nz][nx]. */
af_status af_backward(af_ctx* ctx, const af_complex* iq_dev, const af_loss_params* lp,
                const af_complex* gblk_dev, float* grad_dev);

/* One plain-method iteration: the loss at s_dev (terms_dev), its gradient (the
 * same passes as af_loss_and_grad), then an Adam step (the paper's Eq. 9 uses
 * plain descent; Adam replaces it here) updating s_dev, m_dev, v_dev ([nz][nx],
 * device, in place).  step is 1-based.  The context's slowness becomes the
 * updated s. */
af_status af_autofocus_step(af_ctx* ctx, const af_complex* iq_dev, const af_loss_params* lp,
                      const af_adam_params* ap, int step, float* s_dev, float* m_dev,
                      float* v_dev, float* terms_dev);

/* Dynamic CMPE grid of the global-speed initialisation (Section II-C, Sound Speed
 * Estimation; Section III-A): the pixels of af_set_geometry are taken as laid out
 * for the speed c_ref (mm/us).  At a sweep speed c_g every pixel's depth below the
 * physical lens surface is stretched by c_g / c_ref -- along its polar angle for a
 * curvilinear array, straight down for a linear one -- and the patch spacing
 * becomes c_g / (2 fc) (lambda_g / 2), so the same time samples stay under each
 * pixel.  Speeds may range over [c_min, c_max].  The pixel-to-tile assignment of
 * af_set_geometry is kept; the context then needs af_set_slowness again, with a
 * grid that covers the points at every speed of the range (AF_ERR_STATE until
 * then).
 * A later af_set_geometry ends the dynamic grid.
 * Errors: AF_ERR_STATE before geometry and lens; AF_ERR_ARG for c_ref, fc or c_min
 * not positive, or c_max < c_min. */
af_status af_set_dynamic_grid(af_ctx* ctx, double c_ref, double fc, double c_min, double c_max);

/* Moves the dynamic grid's points to speed c_g on the device (positions, active
 * element ranges of Eq. 4, tile ranges), reads the tiles' ranges back (the stream
 * is synchronised) and rebuilds the work lists.  The slowness is not changed.
 * Errors: AF_ERR_STATE without a dynamic grid; AF_ERR_ARG for c_g outside
 * [c_min, c_max] or a point whose active elements are not contiguous (the context
 * then needs af_set_geometry again); AF_ERR_OOM. */
af_status af_set_sweep_speed(af_ctx* ctx, double c_g);

/* Global-speed sweep of the model initialisation (Section II-C): for each of the n
 * speeds (host array, within the dynamic grid's range) the CMPE of the uniform
 * slowness 1/c_g, on the dynamic grid of c_g (dynamic != 0) or on the one grid of
 * static_c for every speed (dynamic = 0, the static grid it replaces).  cmpe_dev:
 * float[n] (device).  *best (host) is the speed of the lowest CMPE, the first one
 * on ties; the context is left on the grid of the best speed (dynamic) or the
 * static grid, with the uniform slowness 1/best.  Synchronises the stream once per
 * speed (af_set_sweep_speed) and at the end.
 * Errors: AF_ERR_STATE without geometry, lens, slowness or dynamic grid;
 * AF_ERR_ARG for n < 1, null pointers, or speeds outside the range. */
af_status af_sweep(af_ctx* ctx, const af_complex* iq_dev, const af_loss_params* lp, int n,
                   const double* speeds, int dynamic, double static_c, float* cmpe_dev,
                   double* best);

/* One-way travel times T[a][p] (us) at the current slowness, caller point
 * order, float32 [n_elem][P] (device); entries outside the apodisation are NaN. */
af_status af_travel_times(af_ctx* ctx, float* t_dev);

/* Channel-data simulator: point scatterers in a true slowness map, echoes at the
 * bent-ray round-trip times (same ray model, `n_seg` segments, refraction at the
 * node-mean speed), baseband Gaussian envelope of -6 dB fractional bandwidth
 * frac_bw truncated at 6 sigma, phase exp(-j 2 pi fd tau).  Uses the geometry,
 * lens and acquisition of af_set_geometry / af_set_lens.  The echoes are summed
 * in 64-bit fixed point (2^-32), so the output repeats bit for bit from run to
 * run; records of up to 10240 samples, and the sum of |amp| below 2^31
 * (AF_ERR_ARG otherwise, also for amplitudes that are not finite).
 *   scat_xz [n_scat][2] float64, amp [n_scat] float32 (host);
 *   s_true_dev [nz][nx] float32 (device) on the node grid (x0, z0, dx, dz);
 *   iq_dev [n_elem][n_elem][n_samples] output (device, overwritten). */
af_status af_simulate(af_ctx* ctx, int n_scat, const double* scat_xz, const float* amp,
                int nx, int nz, double x0, double z0, double dx, double dz,
                const float* s_true_dev, int n_seg, double fc, double frac_bw,
                af_complex* iq_dev);

/* ---- Learned warm start: BF16 matrix-core 3x3 convolutions ------------------------
 * Layer of the small CNN that predicts a slowness map from features of a
 * homogeneous beamform.  Convolutions are 3x3, padding 1, stride 1 or 2, tensors
 * NHWC; activations and packed weights are BF16 (raw 16-bit words), accumulation
 * FP32.  Ho = (H - 1) / stride + 1, likewise Wo.  Kp = 9 Cin and Ktp = 9 Cout,
 * each rounded up to a multiple of 16.  All pointers are device pointers; every
 * call only enqueues on the context stream.  These calls need no geometry.
 * Activation pointers are 16-byte aligned when their channel count is a multiple
 * of 8 (8-byte when a multiple of 4).
 * Errors: AF_ERR_ARG for Cin or Cout outside 1..32, stride not 1 or 2, non-
 * positive sizes, activations of 2 GiB or more (B H W max(Cin, Cout) BF16 values)
 * or a null required pointer. */

/* Packs FP32 weights w[Cout][3][3][Cin] into the BF16 operands of the forward,
 * wpack [32][Kp] (row = output channel), and of the backward-data pass, wtpack
 * [32][Ktp] (row = input channel, column = tap * Cout + co); zero padding.
 * wtpack may be NULL. */
af_status af_conv3x3_pack(af_ctx* ctx, int Cin, int Cout, const float* w, void* wpack,
                          void* wtpack);
/* out = act(conv(in, w) + bias): in [B][H][W][Cin] BF16, bias [Cout] FP32;
 * out_bf16 [B][Ho][Wo][Cout] BF16 after ReLU if relu != 0 (may be NULL);
 * out_f32 the same before ReLU in FP32 (may be NULL). */
af_status af_conv3x3_fwd(af_ctx* ctx, int B, int H, int W, int Cin, int Cout, int stride,
                         int relu, const void* in_bf16, const void* wpack, const float* bias,
                         void* out_bf16, float* out_f32);
/* din [B][H][W][Cin] BF16 = transposed convolution of dout [B][Ho][Wo][Cout] BF16
 * with the weights, times the ReLU mask act > 0 of the layer below when act_bf16
 * ([B][H][W][Cin], that layer's output) is not NULL. */
af_status af_conv3x3_bwd_data(af_ctx* ctx, int B, int H, int W, int Cin, int Cout, int stride,
                              const void* dout_bf16, const void* wtpack, const void* act_bf16,
                              void* din_bf16);
/* dw [Cout][3][3][Cin] and dbias [Cout] (FP32, overwritten) from the layer input
 * in_bf16 and dout_bf16.  Split over pixels, partial sums reduced in fixed order. */
af_status af_conv3x3_bwd_weight(af_ctx* ctx, int B, int H, int W, int Cin, int Cout, int stride,
                                const void* in_bf16, const void* dout_bf16, float* dw,
                                float* dbias);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight training or serving loops, harnesses that forbid hipMalloc): the same
 * result as af_conv3x3_bwd_weight, bit for bit (the same kernels in the same
 * order), with its partial sums in a static device array of the library instead
 * of a buffer the context allocates on first use.  The array holds 800 x 9248
 * floats (29.6 MB) on every GPU the library runs on, until the process ends; that
 * is what any valid shape needs, and a larger need is rejected with AF_ERR_ARG.
 * The call allocates nothing.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, threads or contexts) race.
 * Errors: those of af_conv3x3_bwd_weight; AF_ERR_HIP if af_create could not take
 * the array's address on this device. */
af_status af_conv3x3_bwd_weight_noalloc(af_ctx* ctx, int B, int H, int W, int Cin, int Cout,
                                        int stride, const void* in_bf16, const void* dout_bf16,
                                        float* dw, float* dbias);
/* Squared error: loss_parts[ceil(n/256)] = block sums of scale (out - label)^2 and
 * dout_bf16[n] = 2 scale (out - label). */
af_status af_mse_loss(af_ctx* ctx, int n, const float* out, const float* label, float scale,
                      float* loss_parts, void* dout_bf16);
/* Adam (with bias correction) on n FP32 parameters p with moments m, v and gradient g. */
af_status af_adam_update(af_ctx* ctx, int n, const af_adam_params* ap, int step, float* p,
                         float* m, float* v, const float* g);
/* NHWC BF16 network input from C channel-major FP32 maps [C][n]:
 * out[i][c] = bf16((maps[c][i] - shift[c]) * scale[c]), the difference and product
 * in FP32, rounded to BF16 to nearest even (shift, scale: device, C floats). */
af_status af_features(af_ctx* ctx, long long n, int C, const float* maps, const float* shift,
                      const float* scale, void* out_bf16);
/* Slowness grid [nz][nx] (node (i, j) at (x0 + j dx, z0 + i dz)) from a polar map
 * [nr][nt] (rows: radius r0 + a dr; columns: polar angle t0 + b dt, angles from
 * the z axis towards x):  with u = (|node| - r0)/dr and v = (angle - t0)/dt, each
 * clamped to the map's index range, s = s_base + scale * (bilinear interpolation
 * of the map at (u, v)), then clamped to [s_lo, s_hi] (a non-finite value gives
 * s_lo), so a network output always yields a slowness the hot path accepts.
 * Errors: AF_ERR_ARG for nr or nt < 2, non-positive sizes or steps, or
 * 0 < s_lo <= s_hi violated. */
af_status af_polar_to_grid(af_ctx* ctx, const float* map, int nr, int nt, double r0, double dr,
                           double t0, double dt, int nx, int nz, double x0, double z0,
                           double dx, double dz, float s_base, float scale, float s_lo,
                           float s_hi, float* s_dev);

/* Kernel timing with HIP events on the context stream.  While enabled, each
 * kernel of the loss, gradient and update calls and each convolution call (the
 * weight gradient counts its partial-sum reduce with it) is bracketed by two
 * events; af_profile_read waits for the stream, returns the summed milliseconds
 * and launch counts per kernel family (arrays of AF_K_COUNT entries, host) and
 * clears the record. */
enum {
  AF_K_PREPARE = 0, AF_K_TABLE = 1, AF_K_DAS_FWD = 2, AF_K_CMPE = 3, AF_K_FINALIZE = 4,
  AF_K_GSCALE = 5, AF_K_DAS_ADJ = 6, AF_K_PATH_ADJ = 7, AF_K_FOLD = 8, AF_K_ADAM = 9,
  AF_K_EXPORT = 10, AF_K_CONV_FWD = 11, AF_K_CONV_BWD_DATA = 12, AF_K_CONV_BWD_WEIGHT = 13,
  AF_K_COUNT = 14
};
af_status af_set_profiling(af_ctx* ctx, int enable);
af_status af_profile_read(af_ctx* ctx, double* ms, long long* calls);

/* Sizes and diagnostics. */
enum {
  AF_Q_P = 0,            /* caller points n_pix * patch^2 */
  AF_Q_P_INTERNAL = 1,   /* internal (tiled, padded) points */
  AF_Q_NBLK = 2,         /* blocks per aperture */
  AF_Q_GBLK_ELEMS = 3,   /* complex elements of gblk_dev for af_forward */
  AF_Q_ACTIVE_PAIRS = 4, /* sum over points of active elements (rays) */
  AF_Q_ACTIVE_SAMPLES = 5, /* sum over points of active (t, r) pairs */
  AF_Q_TILES = 6,
  AF_Q_NA_MAX = 7,       /* largest active element range of a tile */
  AF_Q_NBA_MAX = 8,      /* largest active block range of a tile */
  AF_Q_WIDE_TILES = 9,   /* tiles whose CMPE stage runs from device memory */
  AF_Q_CHUNKS = 10,      /* chunks of tiles the hot path runs over (1 without a budget) */
  AF_Q_DEVICE_BYTES = 11 /* device memory the context holds */
};
af_status af_query(af_ctx* ctx, int what, long long* out);

#ifdef __cplusplus
}
#endif
#endif /* AF_H_ */
