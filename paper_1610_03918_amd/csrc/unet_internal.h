// Internal interface of the learned warm start: the U-Net kernels
// (unet_kernels.hip) and the host runtime behind pic_unet.h (unet_runtime.cpp).
//
// Tensors are NHWC: pixel (b, h, w) of an H x W image at ((b*H + h)*W + w),
// channels innermost.  Activations are bfloat16 (stored as uint16_t),
// gradients flowing between layers float32, parameters float32 masters with
// bfloat16 copies laid out for the matrix cores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace unet {

constexpr int kLevels = 4;
constexpr int kNConv = 14;                 // 8 encoder/bottleneck + 6 decoder
constexpr int kInCh = 3;
constexpr int kKChunk = 32;                // channels per K step of the convolutions

__host__ __device__ inline int pad32(int c) { return (c + 31) & ~31; }

// One convolution (forward or input gradient) as an implicit GEMM.
struct ConvArgs {
    int B, H, W;                 // output pixels (= full-resolution input pixels)
    const uint16_t *src;         // full-resolution input [B,H,W,Cs]: channels Cu .. Cu+Cs-1
    int Cs;
    const uint16_t *up;          // half-resolution input [B,H/2,W/2,Cu], upsampled by copying
    int Cu;                      //   each pixel to a 2x2 block: channels 0 .. Cu-1 (may be 0)
    int Cin_pad;                 // weight row length (multiple of 32)
    const uint16_t *wt;          // [Cout][9][Cin_pad], tap t = 3*dh + dw
    const float *bias;           // [Cout] (forward only; rounded to bfloat16 like the weights)
    int Cout;                    // multiple of 16
    void *out;                   // forward: bf16 [P][Cout] after bias + ReLU; gradient: f32 [P][Cout]
    int pw;                      // 1: the image wraps along W (circular padding), 0: zero padding
};

// Weight gradient of one convolution, split over pixel tiles.
struct WgradArgs {
    int B, H, W;
    const uint16_t *gy;          // output gradient after the ReLU mask, bf16 [P][Cout]
    int Cout;
    const uint16_t *src;         // the convolution's input, as in ConvArgs
    int Cs;
    const uint16_t *up;
    int Cu;
    int Cin_pad;
    int nsplit;
    float *part;                 // [nsplit][Cout][9][Cin_pad]
    float *bpart;                // [nsplit][Cout]
    int pw;                      // as in ConvArgs
};

// Gradient through a ReLU (and the skip / pooling / upsampling joins):
//   gy[p][c] = bf16((A(p,c) + B(p,c)) * [h[p][c] > 0])
// A: a_up == 0: ga[p*sa + oa + c];  a_up == 1: sum of ga over the 2x2 block
//    of p at the finer level (the adjoint of upsampling by copying);
// B: gb == null: 0; else 0.25 * gb[parent(p)*C + c] at the coarser level
//    (the adjoint of 2x2 averaging).
struct ReluBwdArgs {
    int B, H, W, C;              // level of gy / h
    const float *ga;
    int sa, oa, a_up;
    const float *gb;
    const uint16_t *h;
    uint16_t *gy;
};

void launch_conv(const ConvArgs &a, bool f32out, hipStream_t s);
void launch_wgrad(const WgradArgs &a, int ci_chunks, hipStream_t s);
int wgrad_tiles(int B, int H, int W);
void launch_wgrad_reduce(const float *part, const float *bpart, int nsplit, int Cout, int Cin,
                         int Cin_pad, float *gw, float *gb, hipStream_t s);
void launch_pool(const uint16_t *in, uint16_t *out, int B, int H, int W, int C, hipStream_t s);
void launch_relu_bwd(const ReluBwdArgs &a, hipStream_t s);
void launch_head_fwd(const uint16_t *h, const float *wh, float *out, long long P, hipStream_t s);
// gy = bf16(gout * wh * [h > 0]); per-block partial sums of gout * h (16) and gout (1)
int head_bwd_blocks(long long P);
void launch_head_bwd(const uint16_t *h, const float *wh, const float *gout, uint16_t *gy,
                     double *part, long long P, hipStream_t s);
void launch_head_finalize(const double *part, int nblk, float *gwh, hipStream_t s);
int loss_blocks(long long P);
void launch_mask_sum(const float *mask, double *part, long long P, hipStream_t s);
void launch_loss(const float *out, const float *target, const float *mask, const double *msum,
                 float *gout, double *part, long long P, hipStream_t s);
void launch_sum_parts(const double *part, int n, double *dst, hipStream_t s);
void launch_wprep(const float *w, int Cin, int Cout, uint16_t *wf, uint16_t *wd, hipStream_t s);
void launch_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s);
void launch_snapshot(const double *b, const double *phi, const uint8_t *node_cond, int NX, int NY,
                     int H, int W, float s_rho, float s_v, float s_phi, uint16_t *x, float *target,
                     float *mask, hipStream_t s);
void launch_guess(const float *out, const double *b, const uint8_t *node_cond, int NX, int NY,
                  int H, int W, float s_phi, double *guess, hipStream_t s);
// residual learning (see pic_unet.h: pic_unet_residual_sample, pic_unet_load, pic_unet_residual_guess)
// stats (may be null) += deterministic sums over the window; part: 3 doubles per
// block of rsample_blocks(H, W) (needed only with stats)
long long rsample_blocks(int H, int W);
void launch_rsample(const double *b, const double *p1, const double *p2, const double *pt,
                    const uint8_t *nc, int NX, int NY, int px, int py, int H, int W, float s_r, float s_v,
                    float s_d, uint16_t *x, uint16_t *t, double *stats, double *part, hipStream_t s);
// The same with the partial sums in the library's static device scratch
// (no work array); with stats, windows of at most rsample_static_max_pixels().
long long rsample_static_max_pixels();
hipError_t launch_rsample_static(const double *b, const double *p1, const double *p2, const double *pt,
                                 const uint8_t *nc, int NX, int NY, int px, int py, int H, int W, float s_r,
                                 float s_v, float s_d, uint16_t *x, uint16_t *t, double *stats, hipStream_t s);
void launch_load(const uint16_t *xs, const uint16_t *ts, long long P, uint16_t *x, float *target, float *mask,
                 hipStream_t s);
void launch_rguess(const float *out, const double *p1, const double *p2, const uint8_t *nc, int NX, int NY,
                   int H, int W, float s_d, int use_out, double *guess, hipStream_t s);
// time extrapolation of the potential: out = sum_k c[k] p[k] (k in order)
constexpr int kExtrapMax = 8;
struct ExtrapArgs {
    const double *p[kExtrapMax];
    double c[kExtrapMax];
    int K;
    long long n;
    double *out;
};
void launch_extrapolate(const ExtrapArgs &a, hipStream_t s);
// coarse residual learning (pixel = f x f block of nodes, f divides 16):
// the sample (part: 3 float64 per block of csample_blocks(f, H, W), needed
// only with stats) and the prolonged start
long long csample_blocks(int f, int H, int W);
void launch_csample(const double *b, const double *p1, const double *p2, const double *pt, const uint8_t *nc,
                    int NX, int NY, int px, int py, int f, int H, int W, float s_r, float s_v, float s_d,
                    uint16_t *x, uint16_t *t, double *stats, double *part, hipStream_t s);
void launch_cguess(const float *out, const double *p1, const double *p2, const uint8_t *nc, int NX, int NY,
                   int px, int py, int f, int H, int W, float s_d, int use_out, double *guess, hipStream_t s);

} // namespace unet
