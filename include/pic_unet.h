/*
 * pic_unet.h - C ABI of the learned warm start for the field solve of
 * eq. (5) (arXiv:1610.03918, Sec. II).  The paper names the field solver as
 * the part of the cycle whose speed matters most (Sec. IV); this library
 * starts the Poisson solve from the prediction of a small convolutional
 * network and always finishes it with the ordinary solver to the requested
 * tolerance, so the result does not depend on the prediction beyond that
 * tolerance.
 *
 * Network: a 4-level U-Net.  Level l (0..3) works on (H >> l) x (W >> l)
 * pixels with 16 << l channels: two 3x3 convolutions with zero padding and
 * ReLU per level, 2x2 average pooling between encoder levels, copying
 * (nearest-neighbour) upsampling, concatenation [upsampled, skip] before the
 * first decoder convolution of a level, and a 1x1 head (16 -> 1, float32).
 * Weights and activations are bfloat16, products accumulate in float32.
 *
 * Tensors are NHWC: pixel (b, h, w) at ((b*H + h)*W + w).  Pixel (h, w)
 * stands for node (h, w) of the Poisson grid (NX x NY nodes, row-major in x;
 * H <= NX and W <= NY, both multiples of 8).  Input channels: 0 the source
 * term on free nodes times s_rho, 1 a free-node indicator, 2 the Dirichlet
 * value times s_v on conductor nodes.  Output: phi / s_phi.
 *
 * Parameters: one float32 array of pic_unet_param_count() values.  For each
 * 3x3 convolution k = 0..13 in network order (encoder levels 0..3, then the
 * decoder levels 2, 1, 0) the weight [Cout][3][3][Cin] (tap row along H)
 * followed by the bias [Cout]; then the head weight [16] and bias [1].
 * pic_unet_layer reports the shapes and offsets.
 *
 * Ownership: the caller allocates parameters, gradients, the two Adam
 * moment arrays (each param_count float32, device) and one workspace of
 * pic_unet_workspace_size bytes, and keeps them alive until
 * pic_unet_destroy.  The library never allocates device memory.  Calls are
 * enqueued on the stream given at creation and return without waiting unless
 * stated.  Errors: a pic_status; pic_unet_last_error explains.  Not thread
 * safe.
 */
#ifndef PIC_UNET_H
#define PIC_UNET_H

#include "pic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pic_unet pic_unet;

#define PIC_UNET_NCONV 14

typedef struct {
    int32_t cin, cout;           /* channels (the head: 16, 1) */
    int32_t level;               /* resolution level 0..3 */
    int32_t pad;
    int64_t w_offset, b_offset;  /* offsets (float32 values) into the parameter array */
} pic_unet_layer;

typedef struct {
    uint16_t *input;             /* bfloat16 [B][H][W][3] */
    float *output;               /* [B][H][W] (phi / s_phi) */
    float *target;               /* [B][H][W] training target (phi / s_phi) */
    float *mask;                 /* [B][H][W] loss weight (1 on free nodes) */
    float *grad_output;          /* [B][H][W] d loss / d output */
} pic_unet_io;

/* Number of float32 parameters. */
int64_t pic_unet_param_count(void);

/* Shape and offsets of convolution k (0..13) or of the head (k = 14). */
pic_status pic_unet_layer_info(int32_t k, pic_unet_layer *out);

/* Workspace bytes for batch B of H x W images (H, W multiples of 8). */
pic_status pic_unet_workspace_size(int32_t batch, int32_t H, int32_t W, size_t *bytes);

/* Creates a network over caller-owned device arrays (see Ownership).  The
 * parameters are read at the first forward pass (and after
 * pic_unet_params_changed); the Adam moments must start at zero. */
pic_status pic_unet_create(int32_t batch, int32_t H, int32_t W, float *params, float *grads,
                           float *adam_m, float *adam_v, void *workspace, size_t workspace_bytes,
                           void *stream, pic_unet **out);

/* Device pointers of the input/output tensors inside the workspace. */
pic_status pic_unet_io_buffers(pic_unet *u, pic_unet_io *io);

/* The caller rewrote the parameter array: re-derive the bfloat16 copies. */
pic_status pic_unet_params_changed(pic_unet *u);

/* input -> output for the whole batch (keeps the activations for backward). */
pic_status pic_unet_forward(pic_unet *u);

/* Masked mean-square loss sum(mask (output - target)^2) / sum(mask) over
 * the batch, and grad_output.  Waits; *loss (may be NULL) receives it. */
pic_status pic_unet_loss(pic_unet *u, double *loss);

/* grad_output -> gradients of every parameter (overwrites the gradient
 * array).  Needs the activations of the last pic_unet_forward. */
pic_status pic_unet_backward(pic_unet *u);

/* One Adam step (bias-corrected moments) on the parameters from the
 * gradients; counts its own steps. */
pic_status pic_unet_adam(pic_unet *u, float lr, float beta1, float beta2, float eps);

/* Writes batch slot `slot` of the input from a Poisson problem: b (device
 * NX*NY float64, the assembled right-hand side whose Dirichlet nodes hold
 * their potentials) and node_cond (device NX*NY, see pic_node_map).  If phi
 * (device NX*NY float64) is not NULL also the target (phi / s_phi) and the
 * mask (free nodes) of that slot. */
pic_status pic_unet_snapshot(pic_unet *u, int32_t slot, const double *b, const double *phi,
                             const uint8_t *node_cond, int32_t NX, int32_t NY, float s_rho,
                             float s_v, float s_phi);

/* Writes guess (device NX*NY float64): output of `slot` times s_phi on free
 * nodes inside the H x W window, 0 on free nodes outside it, b on Dirichlet
 * nodes - a start for pic_solve(ctx, 2, guess, ...). */
pic_status pic_unet_guess(pic_unet *u, int32_t slot, const double *b, const uint8_t *node_cond,
                          int32_t NX, int32_t NY, float s_phi, double *guess);

/* Learned start of instance 0 of ctx (batch slot 0 of u) that predicts phi
 * itself: snapshot of the current right-hand side b (the caller's
 * pic_buffers.b), forward pass, guess into the caller's device scratch
 * guess (NX*NY float64), then pic_solve(ctx, 2, guess, info).  The
 * network's stream first waits for the work queued on the context's
 * stream.  Waits (as pic_solve).  (The residual form below is the one the
 * solver uses.) */
pic_status pic_solve_learned(pic_ctx *ctx, pic_unet *u, const double *b, float s_rho, float s_v,
                             float s_phi, double *guess, pic_solve_info *info);

/* ---- residual learning: the start used with the plain solver ----------
 * The network corrects the linear extrapolation in time of the potential,
 * phi_s = 2 phi_1 - phi_2 (phi_1, phi_2 the solutions of the two previous
 * steps; phi_1 alone when phi_2 is NULL), the start the solver already uses
 * (pic_solve guess kind 3).  Input channels: 0 the residual r = b - A phi_s
 * of eq. (5)'s 5-point system on free nodes times s_r, 1 the free-node
 * indicator, 2 the Dirichlet value times s_v on conductor nodes.  Target:
 * (phi - phi_s) s_d on free nodes.  The start is phi_s + output / s_d. */

/* Circular padding of every convolution along W (periodic_w = 1) for a
 * grid periodic along y whose node count NY equals the network's W; 0
 * (the default) pads with zeros.  PIC_ERR_ARG for other values. */
pic_status pic_unet_set_periodic(pic_unet *u, int32_t periodic_w);

/* Bytes of the work array pic_unet_residual_sample needs for an H x W
 * window when it returns statistics: 3 float64 per block of 256 pixels. */
pic_status pic_unet_residual_sample_work_bytes(int32_t H, int32_t W, size_t *bytes);

/* One training sample of the H x W window of a Poisson problem (no network
 * needed): x (device bfloat16 [H][W][3]) receives the input channels above,
 * t (device bfloat16 [H][W], or NULL) the target with phi_t the converged
 * potential.  stats (device float64[3], or NULL) accumulates the sums over
 * the window's free nodes of r^2 and of (phi_t - phi_s)^2 and their count,
 * added in a fixed order (deterministic); with stats, work (device, at
 * least pic_unet_residual_sample_work_bytes) holds the per-block partial
 * sums.  b, phi_1, phi_2 (may be NULL), phi_t: device float64 NX x NY;
 * node_cond: device NX x NY node map (0 free); periodic_x / periodic_y: the
 * grid's periodic axes (neighbours wrap).  Enqueued on stream.  PIC_ERR_ARG
 * for a window larger than the grid, a missing pointer or a short work
 * array. */
pic_status pic_unet_residual_sample(const double *b, const double *phi_1, const double *phi_2,
                                    const double *phi_t, const uint8_t *node_cond, int32_t NX, int32_t NY,
                                    int32_t periodic_x, int32_t periodic_y, int32_t H, int32_t W, float s_r,
                                    float s_v, float s_d, uint16_t *x, uint16_t *t, double *stats,
                                    void *work, size_t work_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sample and statistics as pic_unet_residual_sample, bit for bit, without
 * the work array.  The per-block partial sums live in a static device array
 * of the library (384 KiB per device, held until the process ends), so
 * with stats the window may hold at most 4,194,304 pixels (H * W; 16384
 * blocks of 256): larger windows return PIC_ERR_CAPACITY and launch
 * nothing.  The stream must belong to the current device (PIC_ERR_ARG
 * otherwise).  Allocates nothing.  Every call on a device shares that
 * device's array: calls that overlap on one device (two streams, or two
 * host threads) race and must be serialised by the caller. */
pic_status pic_unet_residual_sample_noalloc(const double *b, const double *phi_1, const double *phi_2,
                                            const double *phi_t, const uint8_t *node_cond, int32_t NX,
                                            int32_t NY, int32_t periodic_x, int32_t periodic_y, int32_t H,
                                            int32_t W, float s_r, float s_v, float s_d, uint16_t *x, uint16_t *t,
                                            double *stats, void *stream);

/* Copies a stored sample (x, t as written by pic_unet_residual_sample for
 * this network's H x W) into batch slot `slot`: the input, and with t the
 * training target (as float32) and the loss mask (the free-node channel). */
pic_status pic_unet_load(pic_unet *u, int32_t slot, const uint16_t *x, const uint16_t *t);

/* Time extrapolation of the potential, the start the network corrects (the
 * paper names no time stencil): out = coef[0] phi[0] + coef[1] phi[1] + ...
 * + coef[K-1] phi[K-1] at each of the n nodes, added in this order in
 * float64 (no fused multiply-add).  phi: host array of K device float64
 * arrays (phi[0] the latest solution, phi[k] the one k steps before), coef:
 * host array of K coefficients, 1 <= K <= 8; out: device float64[n] (may not
 * alias phi).  The K-point polynomial extrapolation to the next step takes
 * coef[k-1] = (-1)^(k+1) binomial(K, k): K = 2 is 2 phi_1 - phi_2, K = 4 is
 * 4 phi_1 - 6 phi_2 + 4 phi_3 - phi_4 (exact for potentials that are
 * polynomials of degree below K in time).  The sample and guess calls take
 * such a start s as phi_1 = phi_2 = s (2 s - s = s exactly).  Enqueued on
 * stream.  PIC_ERR_ARG for K outside 1..8, a negative n or a missing
 * pointer. */
pic_status pic_unet_extrapolate(const double *const *phi, const double *coef, int32_t K, int64_t n, double *out,
                                void *stream);

/* Writes guess (device float64 NX x NY): phi_s plus output(slot) / s_d on
 * the free nodes of the H x W window (use_output = 0: phi_s alone, the plain
 * extrapolation), phi_s on every other node - a start for pic_solve(ctx, 2
 * or 4, guess, ...), which reads its free nodes only. */
pic_status pic_unet_residual_guess(pic_unet *u, int32_t slot, const double *phi_1, const double *phi_2,
                                   const uint8_t *node_cond, int32_t NX, int32_t NY, float s_d,
                                   int32_t use_output, double *guess);

/* Learned start of instance 0 of a running simulation ctx (batch slot 0 of
 * u): the sample of the context's current b, its current potential (phi_1)
 * and the solution before it (phi_2, when a kind-3 or kind-4 solve has run),
 * a forward pass, the corrected start into the caller's device scratch
 * guess (NX*NY float64), then pic_solve(ctx, 4, guess, info), which keeps
 * the time history for the next extrapolation.  The network's stream first
 * waits for the work queued on the context's stream.  Waits (as
 * pic_solve). */
pic_status pic_solve_learned_residual(pic_ctx *ctx, pic_unet *u, float s_r, float s_v, float s_d,
                                      double *guess, pic_solve_info *info);

/* ---- coarse residual learning: the start the benchmark's learned solve uses ----
 * The solver's iteration count is set by the smooth part of its start's
 * error, whose extent is the whole grid; a network that sees one node per
 * pixel reaches only its receptive field (tens of nodes).  Here pixel
 * (h, w) stands for the f x f block of nodes (h f + p, w f + q), p, q < f,
 * f one of 1, 2, 4, 8, 16, covering H f <= NX by W f <= NY nodes.  Input
 * channels: 0 the mean over the block of the residual r = b - A phi_s of
 * the extrapolated start (zero on Dirichlet nodes) times s_r, 1 the
 * fraction of free nodes in the block, 2 the mean of the Dirichlet values
 * (zero on free nodes) times s_v.  Target: the block mean of (phi - phi_s)
 * on free nodes times s_d.  Each mean adds the block's nodes in row-major
 * order from zero, then multiplies by 1/f^2; values are rounded to bfloat16.
 * The start adds to phi_s, on every free node of the covered region, c / s_d
 * with c the bilinear interpolation of the output at the node's pixel
 * coordinate ((i + 1/2)/f - 1/2, (j + 1/2)/f - 1/2): an axis that is
 * periodic and covered exactly (H f = NX, W f = NY) wraps, any other is held
 * at its edge pixels; nodes outside the covered region start from phi_s.
 * f = 1 gives pic_unet_residual_sample / pic_unet_residual_guess. */
/* Bytes of the work array of pic_unet_coarse_sample with statistics. */
pic_status pic_unet_coarse_sample_work_bytes(int32_t f, int32_t H, int32_t W, size_t *bytes);
/* One coarse training sample (no network needed): x (device bfloat16
 * [H][W][3]) the input above, t (device bfloat16 [H][W], or NULL) the
 * target for the converged potential phi_t.  stats (device float64[3], or
 * NULL) accumulates the sums over pixels of (block mean of r)^2 and of
 * (block mean of phi_t - phi_s)^2 and the count of pixels holding a free
 * node, in a fixed order; with stats, work (device, at least
 * pic_unet_coarse_sample_work_bytes) holds per-block partial sums.  Other
 * arguments as pic_unet_residual_sample.  Enqueued on stream.  PIC_ERR_ARG
 * for a factor not listed, a window that does not fit the grid, a missing
 * pointer or a short work array. */
pic_status pic_unet_coarse_sample(const double *b, const double *phi_1, const double *phi_2, const double *phi_t,
                                  const uint8_t *node_cond, int32_t NX, int32_t NY, int32_t periodic_x,
                                  int32_t periodic_y, int32_t f, int32_t H, int32_t W, float s_r, float s_v,
                                  float s_d, uint16_t *x, uint16_t *t, double *stats, void *work,
                                  size_t work_bytes, void *stream);
/* Writes guess (device float64 NX x NY): the start above from the output of
 * batch slot `slot` of a network of H x W pixels (use_output = 0: phi_s
 * alone), a start for pic_solve(ctx, 2 or 4, guess, ...). */
pic_status pic_unet_coarse_guess(pic_unet *u, int32_t slot, const double *phi_1, const double *phi_2,
                                 const uint8_t *node_cond, int32_t NX, int32_t NY, int32_t periodic_x,
                                 int32_t periodic_y, int32_t f, float s_d, int32_t use_output, double *guess);
/* As pic_solve_learned_residual with the coarse sample and start of factor
 * f: the sample of the context's current b and potentials, a forward pass,
 * the prolonged start into guess, then pic_solve(ctx, 4, guess, info).
 * Waits (as pic_solve). */
pic_status pic_solve_learned_coarse(pic_ctx *ctx, pic_unet *u, int32_t f, float s_r, float s_v, float s_d,
                                    double *guess, pic_solve_info *info);
/* HIP-event timing of pic_unet_forward on the library stream (default off);
 * average ms per forward pass since the last read, then reset. */
pic_status pic_unet_set_timing(pic_unet *u, int32_t on);
pic_status pic_unet_forward_timing(pic_unet *u, double *avg_ms, int32_t *passes);

void pic_unet_destroy(pic_unet *u);
const char *pic_unet_last_error(const pic_unet *u);

#ifdef __cplusplus
}
#endif
#endif /* PIC_UNET_H */
