// gfx950 kernels of the learned warm start: a 4-level U-Net (16/32/64/128
// channels, 3x3 convolutions, bfloat16 weights and activations, float32
// accumulation on the matrix cores) with its backward pass, loss, Adam step,
// and the maps between the Poisson problem and the network's tensors.
//
// Convolutions run as implicit GEMMs on v_mfma_f32_16x16x32_bf16: the
// weights are the M operand (output channels), the pixels the N operand and
// the K dimension walks (tap, input channel).  A block stages a
// (rows+2) x 18 pixel patch of 32 input channels and the matching weights in
// LDS, then every wave multiplies 16 x 16 tiles.  The input gradient is the
// same kernel with the taps flipped and the weights transposed; the weight
// gradient contracts over pixels in a split-K kernel whose partial sums are
// added in a fixed order (deterministic).
#include "unet_internal.h"

#include <mutex>

namespace unet {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int KS = 40;           // LDS row length (bf16) of one pixel's 32-channel chunk, padded
constexpr int PC = 18;           // patch columns: 16 output columns + 2 halo

// float32 -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint32_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *(const uint4 *)p);
}
__device__ __forceinline__ bf16x8 pack8(const uint32_t *x) {
    uint4 v = make_uint4(x[0] | (x[1] << 16), x[2] | (x[3] << 16), x[4] | (x[5] << 16),
                         x[6] | (x[7] << 16));
    return __builtin_bit_cast(bf16x8, v);
}

// Stage the input patch rows h0-1 .. h0+PR-2, columns w0-1 .. w0+16, channels
// c0 .. c0+31 of the concatenation [upsampled(up), src] into LDS as
// [row][col][KS] (zeros outside the image and beyond the channel count).
// pw: the image wraps along W, so the columns -1 and W are W-1 and 0 (the
// patch never reaches farther than one column beyond the image).
template <int PR>
__device__ __forceinline__ void stage_patch(uint16_t *sp, const uint16_t *src, int Cs,
                                            const uint16_t *up, int Cu, int b, int H, int W,
                                            int h0, int w0, int c0, int pw) {
    const int Cin = Cu + Cs;
    const int Hh = H >> 1, Wh = W >> 1;
    for (int e = threadIdx.x; e < PR * PC * 4; e += blockDim.x) {
        const int q = e & 3, pix = e >> 2;
        const int r = pix / PC, s = pix - r * PC;
        const int h = h0 - 1 + r;
        int w = w0 - 1 + s;
        if (pw) w = w < 0 ? w + W : (w == W ? 0 : w);
        const int c = c0 + 8 * q;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (h >= 0 && h < H && w >= 0 && w < W && c < Cin) {
            const size_t pu = ((size_t)b * Hh + (h >> 1)) * Wh + (w >> 1);
            const size_t ps = ((size_t)b * H + h) * W + w;
            if (c + 8 <= Cu) {
                v = *(const uint4 *)(up + pu * Cu + c);
            } else if (c >= Cu && c + 8 <= Cin && (Cs & 7) == 0) {
                v = *(const uint4 *)(src + ps * Cs + (c - Cu));
            } else {
                uint32_t x[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int cc = c + k;
                    x[k] = cc < Cu ? up[pu * Cu + cc] : (cc < Cin ? src[ps * Cs + (cc - Cu)] : 0u);
                }
                v = make_uint4(x[0] | (x[1] << 16), x[2] | (x[3] << 16), x[4] | (x[5] << 16),
                               x[6] | (x[7] << 16));
            }
        }
        *(uint4 *)(sp + pix * KS + 8 * q) = v;
    }
}

// ---- convolution (forward: + bias, ReLU, bf16 out; gradient: f32 out) ----
// Block: 4 waves; output tile 4*NR rows x 16 columns x 16*NCO channels.
// Wave w owns rows w*NR .. w*NR+NR-1.
template <int NCO, int NR, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    constexpr int TX = 4 * NR, PR = TX + 2, CT = 16 * NCO;
    __shared__ __align__(16) uint16_t sp[PR * PC * KS];
    __shared__ __align__(16) uint16_t sw[CT * 9 * KS];
    const int tilesW = (a.W + 15) >> 4, tilesH = (a.H + TX - 1) / TX;
    int bid = blockIdx.x;
    const int tw = bid % tilesW;
    bid /= tilesW;
    const int th = bid % tilesH;
    const int b = bid / tilesH;
    const int co0 = blockIdx.y * CT;
    const int h0 = th * TX, w0 = tw * 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;

    f4 acc[NCO][NR];
#pragma unroll
    for (int j = 0; j < NCO; ++j)
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[j][r] = f4{0.f, 0.f, 0.f, 0.f};

    for (int c0 = 0; c0 < a.Cin_pad; c0 += kKChunk) {
        __syncthreads();
        for (int e = threadIdx.x; e < CT * 9 * 4; e += 256) {
            const int q = e & 3, row = e >> 2;          // row = local channel * 9 + tap
            const int co = co0 + row / 9, t = row - (row / 9) * 9;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (co < a.Cout) v = *(const uint4 *)(a.wt + ((size_t)co * 9 + t) * a.Cin_pad + c0 + 8 * q);
            *(uint4 *)(sw + row * KS + 8 * q) = v;
        }
        stage_patch<PR>(sp, a.src, a.Cs, a.up, a.Cu, b, a.H, a.W, h0, w0, c0, a.pw);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int dh = t / 3, dw = t - 3 * (t / 3);
            bf16x8 A[NCO], Bv[NR];
#pragma unroll
            for (int j = 0; j < NCO; ++j) A[j] = ld8(sw + ((16 * j + n) * 9 + t) * KS + 8 * g);
#pragma unroll
            for (int r = 0; r < NR; ++r) Bv[r] = ld8(sp + ((wave * NR + r + dh) * PC + n + dw) * KS + 8 * g);
#pragma unroll
            for (int j = 0; j < NCO; ++j)
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    acc[j][r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[j], Bv[r], acc[j][r], 0, 0, 0);
        }
    }
    // lane holds output channels co0 + 16j + 4g + (0..3) of pixel column n
#pragma unroll
    for (int j = 0; j < NCO; ++j) {
        const int co = co0 + 16 * j + 4 * g;
        if (co >= a.Cout) continue;
        float bb[4] = {0.f, 0.f, 0.f, 0.f};
        if (!F32OUT) {
#pragma unroll
            for (int i = 0; i < 4; ++i) bb[i] = bf2f(f2bf(a.bias[co + i]));
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int h = h0 + wave * NR + r, w = w0 + n;
            if (h >= a.H || w >= a.W) continue;
            const size_t o = (((size_t)b * a.H + h) * a.W + w) * a.Cout + co;
            if (F32OUT) {
                *(f4 *)((float *)a.out + o) = acc[j][r];
            } else {
                uint32_t y[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) y[i] = f2bf(fmaxf(acc[j][r][i] + bb[i], 0.f));
                *(uint2 *)((uint16_t *)a.out + o) = make_uint2(y[0] | (y[1] << 16), y[2] | (y[3] << 16));
            }
        }
    }
}

template <int NCO, int NR>
static void conv_variant(const ConvArgs &a, bool f32out, hipStream_t s) {
    constexpr int TX = 4 * NR;
    const int tilesW = (a.W + 15) >> 4, tilesH = (a.H + TX - 1) / TX;
    dim3 grid(a.B * tilesH * tilesW, (a.Cout + 16 * NCO - 1) / (16 * NCO));
    if (f32out) hipLaunchKernelGGL((k_conv<NCO, NR, true>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_conv<NCO, NR, false>), grid, dim3(256), 0, s, a);
}

void launch_conv(const ConvArgs &a, bool f32out, hipStream_t s) {
    if (a.Cout % 64 == 0) conv_variant<4, 2>(a, f32out, s);
    else if (a.Cout % 48 == 0) conv_variant<3, 2>(a, f32out, s);
    else if (a.Cout % 32 == 0) conv_variant<2, 2>(a, f32out, s);
    else conv_variant<1, 4>(a, f32out, s);
}

// ---- weight gradient ------------------------------------------------------
// gw[co][t][ci] = sum over pixels p of gy[p][co] * in(p + tap t)[ci]
// Block (split, co tile, 32-channel chunk) walks pixel tiles of 16 x 16
// (tile = split, split + nsplit, ...).  Wave w owns tile rows 4w .. 4w+3, two
// K steps of 32 pixels (2 rows x 16 columns); lane group g takes row
// 2*step + g/2, columns 8*(g%2) .. +7.  Blocks of chunk 0 also sum gy (bias).
constexpr int kWTX = 16;

template <int NCO>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
    constexpr int PR = kWTX + 2, CT = 16 * NCO, GS = CT + 8;
    constexpr int SP = PR * PC * KS, SG = kWTX * 16 * GS;
    constexpr int RED = CT * 9 * 32;
    constexpr int STAGE_B = 2 * (SP + SG), RED_B = 4 * (RED + CT);
    __shared__ __align__(16) unsigned char smem[STAGE_B > RED_B ? STAGE_B : RED_B];
    uint16_t *sp = (uint16_t *)smem;
    uint16_t *sg = sp + SP;
    const int tilesW = (a.W + 15) >> 4, tilesH = (a.H + kWTX - 1) / kWTX;
    const int ntiles = a.B * tilesH * tilesW;
    const int split = blockIdx.x, co0 = blockIdx.y * CT, c0 = blockIdx.z * kKChunk;
    const bool with_bias = blockIdx.z == 0;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int n = lane & 15, g = lane >> 4;
    const bf16x8 ones = __builtin_bit_cast(bf16x8, make_uint4(0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u));

    f4 acc[NCO][9][2];
    f4 bacc[NCO];
#pragma unroll
    for (int j = 0; j < NCO; ++j) {
        bacc[j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[j][t][0] = acc[j][t][1] = f4{0.f, 0.f, 0.f, 0.f};
    }

    for (int tile = split; tile < ntiles; tile += a.nsplit) {
        const int tw = tile % tilesW, rest = tile / tilesW;
        const int th = rest % tilesH, b = rest / tilesH;
        const int h0 = th * kWTX, w0 = tw * 16;
        __syncthreads();
        for (int e = threadIdx.x; e < kWTX * 16 * (CT / 8); e += 256) {
            const int q = e % (CT / 8), px = e / (CT / 8);
            const int h = h0 + (px >> 4), w = w0 + (px & 15);
            uint4 v = make_uint4(0, 0, 0, 0);
            if (h < a.H && w < a.W)
                v = *(const uint4 *)(a.gy + (((size_t)b * a.H + h) * a.W + w) * a.Cout + co0 + 8 * q);
            *(uint4 *)(sg + px * GS + 8 * q) = v;
        }
        stage_patch<PR>(sp, a.src, a.Cs, a.up, a.Cu, b, a.H, a.W, h0, w0, c0, a.pw);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int R = 4 * wave + 2 * ks + (g >> 1);
            const int col0 = 8 * (g & 1);
            bf16x8 A[NCO];
#pragma unroll
            for (int j = 0; j < NCO; ++j) {
                uint32_t x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = sg[(R * 16 + col0 + i) * GS + 16 * j + n];
                A[j] = pack8(x);
            }
#pragma unroll
            for (int dh = 0; dh < 3; ++dh) {
#pragma unroll
                for (int cs = 0; cs < 2; ++cs) {
                    uint32_t x[10];
#pragma unroll
                    for (int k = 0; k < 10; ++k) x[k] = sp[((R + dh) * PC + col0 + k) * KS + 16 * cs + n];
#pragma unroll
                    for (int dw = 0; dw < 3; ++dw) {
                        const bf16x8 Bv = pack8(x + dw);
#pragma unroll
                        for (int j = 0; j < NCO; ++j)
                            acc[j][3 * dh + dw][cs] =
                                __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[j], Bv, acc[j][3 * dh + dw][cs], 0, 0, 0);
                    }
                }
            }
            if (with_bias) {
#pragma unroll
                for (int j = 0; j < NCO; ++j)
                    bacc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[j], ones, bacc[j], 0, 0, 0);
            }
        }
    }
    // sum the four waves in a fixed order, then write this split's partial
    __syncthreads();
    float *red = (float *)smem;
    float *bred = red + RED;
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int j = 0; j < NCO; ++j)
#pragma unroll
                for (int t = 0; t < 9; ++t)
#pragma unroll
                    for (int cs = 0; cs < 2; ++cs)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int idx = ((16 * j + 4 * g + i) * 9 + t) * 32 + 16 * cs + n;
                            red[idx] = (w == 0 ? 0.f : red[idx]) + acc[j][t][cs][i];
                        }
            if (with_bias && n == 0) {
#pragma unroll
                for (int j = 0; j < NCO; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int idx = 16 * j + 4 * g + i;
                        bred[idx] = (w == 0 ? 0.f : bred[idx]) + bacc[j][i];
                    }
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < RED; e += 256) {
        const int col = e / 288, rem = e - col * 288;
        const int t = rem >> 5, ci = rem & 31;
        a.part[(((size_t)split * a.Cout + co0 + col) * 9 + t) * a.Cin_pad + c0 + ci] = red[e];
    }
    if (with_bias)
        for (int e = threadIdx.x; e < CT; e += 256) a.bpart[(size_t)split * a.Cout + co0 + e] = bred[e];
}

int wgrad_tiles(int B, int H, int W) {
    return B * ((H + kWTX - 1) / kWTX) * ((W + 15) >> 4);
}

void launch_wgrad(const WgradArgs &a, int ci_chunks, hipStream_t s) {
    if (a.Cout % 32 == 0) {
        dim3 grid(a.nsplit, a.Cout / 32, ci_chunks);
        hipLaunchKernelGGL(k_wgrad<2>, grid, dim3(256), 0, s, a);
    } else {
        dim3 grid(a.nsplit, a.Cout / 16, ci_chunks);
        hipLaunchKernelGGL(k_wgrad<1>, grid, dim3(256), 0, s, a);
    }
}

// Sum of the split partials: a block owns 64 consecutive outputs and splits
// the partials over 4 lanes per output (k = lane, lane + 4, ...), then adds
// the 4 lane sums in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *part, const float *bpart, int nsplit,
                                                      int Cout, int Cin, int Cin_pad, float *gw, float *gb)
{
    __shared__ double sh[4][64];
    const int o = threadIdx.x & 63, q = threadIdx.x >> 6;
    const long long idx = (long long)blockIdx.x * 64 + o;
    const long long total = (long long)Cout * 9 * Cin;
    double s = 0.0;
    if (idx < total) {
        const int ci = (int)(idx % Cin);
        const long long row = idx / Cin;             // co * 9 + t
        for (int k = q; k < nsplit; k += 4) s += part[((size_t)k * Cout * 9 + row) * Cin_pad + ci];
    } else if (idx < total + Cout) {
        const int co = (int)(idx - total);
        for (int k = q; k < nsplit; k += 4) s += bpart[(size_t)k * Cout + co];
    }
    sh[q][o] = s;
    __syncthreads();
    if (q != 0) return;
    s = ((sh[0][o] + sh[1][o]) + sh[2][o]) + sh[3][o];
    if (idx < total) gw[idx] = (float)s;
    else if (idx < total + Cout) gb[idx - total] = (float)s;
}

void launch_wgrad_reduce(const float *part, const float *bpart, int nsplit, int Cout, int Cin,
                         int Cin_pad, float *gw, float *gb, hipStream_t s) {
    const long long n = (long long)Cout * 9 * Cin + Cout;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, part, bpart,
                       nsplit, Cout, Cin, Cin_pad, gw, gb);
}

// ---- 2 x 2 average pooling --------------------------------------------------
__global__ void k_pool(const uint16_t *in, uint16_t *out, int B, int H, int W, int C) {
    const int Ho = H >> 1, Wo = W >> 1, G = C >> 3;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)B * Ho * Wo * G) return;
    const int q = (int)(idx % G);
    long long p = idx / G;
    const int w = (int)(p % Wo);
    p /= Wo;
    const int h = (int)(p % Ho);
    const int b = (int)(p / Ho);
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int dh = 0; dh < 2; ++dh)
#pragma unroll
        for (int dw = 0; dw < 2; ++dw) {
            const uint4 v = *(const uint4 *)(in + (((size_t)b * H + 2 * h + dh) * W + 2 * w + dw) * C + 8 * q);
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[2 * k] += bf2f(u[k] & 0xFFFFu);
                s[2 * k + 1] += bf2f(u[k] >> 16);
            }
        }
    uint32_t y[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) y[k] = f2bf(0.25f * s[k]);
    *(uint4 *)(out + (((size_t)b * Ho + h) * Wo + w) * C + 8 * q) =
        make_uint4(y[0] | (y[1] << 16), y[2] | (y[3] << 16), y[4] | (y[5] << 16), y[6] | (y[7] << 16));
}

void launch_pool(const uint16_t *in, uint16_t *out, int B, int H, int W, int C, hipStream_t s) {
    const long long n = (long long)B * (H >> 1) * (W >> 1) * (C >> 3);
    hipLaunchKernelGGL(k_pool, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, in, out, B, H, W, C);
}

// ---- gradient through ReLU and the joins ------------------------------------
__global__ void k_relu_bwd(ReluBwdArgs a) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long total = (long long)a.B * a.H * a.W * a.C;
    if (idx >= total) return;
    const int c = (int)(idx % a.C);
    long long p = idx / a.C;
    const int w = (int)(p % a.W);
    const long long bh = p / a.W;
    const int h = (int)(bh % a.H);
    const int b = (int)(bh / a.H);
    float s;
    if (!a.a_up) {
        s = a.ga[p * a.sa + a.oa + c];
    } else {
        const int H2 = 2 * a.H, W2 = 2 * a.W;
        s = 0.f;
#pragma unroll
        for (int dh = 0; dh < 2; ++dh)
#pragma unroll
            for (int dw = 0; dw < 2; ++dw)
                s += a.ga[(((size_t)b * H2 + 2 * h + dh) * W2 + 2 * w + dw) * a.sa + a.oa + c];
    }
    if (a.gb) {
        const int Hh = a.H >> 1, Wh = a.W >> 1;
        s += 0.25f * a.gb[(((size_t)b * Hh + (h >> 1)) * Wh + (w >> 1)) * a.C + c];
    }
    a.gy[idx] = (uint16_t)(bf2f(a.h[idx]) > 0.f ? f2bf(s) : 0u);
}

void launch_relu_bwd(const ReluBwdArgs &a, hipStream_t s) {
    const long long n = (long long)a.B * a.H * a.W * a.C;
    hipLaunchKernelGGL(k_relu_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
}

// ---- 1 x 1 head (16 -> 1, float32 weights) ---------------------------------
__global__ void k_head_fwd(const uint16_t *h, const float *wh, float *out, long long P) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const uint4 v0 = *(const uint4 *)(h + p * 16), v1 = *(const uint4 *)(h + p * 16 + 8);
    const uint32_t u[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        s += bf2f(u[k] & 0xFFFFu) * wh[2 * k];
        s += bf2f(u[k] >> 16) * wh[2 * k + 1];
    }
    out[p] = s + wh[16];
}

void launch_head_fwd(const uint16_t *h, const float *wh, float *out, long long P, hipStream_t s) {
    hipLaunchKernelGGL(k_head_fwd, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, h, wh, out, P);
}

constexpr int kRedPx = 4096;     // pixels per block of the reducing kernels

template <int N>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double *dst) {
    __shared__ double sh[N][256];
#pragma unroll
    for (int k = 0; k < N; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
#pragma unroll
            for (int k = 0; k < N; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < N; ++k) dst[k] = sh[k][0];
    }
}

int head_bwd_blocks(long long P) { return (int)((P + kRedPx - 1) / kRedPx); }

__global__ void k_head_bwd(const uint16_t *h, const float *wh, const float *gout, uint16_t *gy,
                           double *part, long long P) {
    double acc[17];
#pragma unroll
    for (int k = 0; k < 17; ++k) acc[k] = 0.0;
    const long long p0 = (long long)blockIdx.x * kRedPx;
    for (long long p = p0 + threadIdx.x; p < p0 + kRedPx && p < P; p += blockDim.x) {
        const float go = gout[p];
        const uint4 v0 = *(const uint4 *)(h + p * 16), v1 = *(const uint4 *)(h + p * 16 + 8);
        const uint32_t u[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
        uint32_t y[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float a0 = bf2f(u[k] & 0xFFFFu), a1 = bf2f(u[k] >> 16);
            acc[2 * k] += (double)go * a0;
            acc[2 * k + 1] += (double)go * a1;
            const uint32_t g0 = a0 > 0.f ? f2bf(go * wh[2 * k]) : 0u;
            const uint32_t g1 = a1 > 0.f ? f2bf(go * wh[2 * k + 1]) : 0u;
            y[k] = g0 | (g1 << 16);
        }
        acc[16] += go;
        *(uint4 *)(gy + p * 16) = make_uint4(y[0], y[1], y[2], y[3]);
        *(uint4 *)(gy + p * 16 + 8) = make_uint4(y[4], y[5], y[6], y[7]);
    }
    block_sum_store<17>(acc, part + 17 * (size_t)blockIdx.x);
}

void launch_head_bwd(const uint16_t *h, const float *wh, const float *gout, uint16_t *gy,
                     double *part, long long P, hipStream_t s) {
    hipLaunchKernelGGL(k_head_bwd, dim3(head_bwd_blocks(P)), dim3(256), 0, s, h, wh, gout, gy, part, P);
}

__global__ void k_head_finalize(const double *part, int nblk, float *gwh) {
    const int k = threadIdx.x;
    if (k >= 17) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[17 * (size_t)b + k];
    gwh[k] = (float)s;
}

void launch_head_finalize(const double *part, int nblk, float *gwh, hipStream_t s) {
    hipLaunchKernelGGL(k_head_finalize, dim3(1), dim3(64), 0, s, part, nblk, gwh);
}

// ---- masked mean-square loss ---------------------------------------------------
int loss_blocks(long long P) { return (int)((P + kRedPx - 1) / kRedPx); }

__global__ void k_mask_sum(const float *mask, double *part, long long P) {
    double acc[1] = {0.0};
    const long long p0 = (long long)blockIdx.x * kRedPx;
    for (long long p = p0 + threadIdx.x; p < p0 + kRedPx && p < P; p += blockDim.x) acc[0] += mask[p];
    block_sum_store<1>(acc, part + blockIdx.x);
}

void launch_mask_sum(const float *mask, double *part, long long P, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_sum, dim3(loss_blocks(P)), dim3(256), 0, s, mask, part, P);
}

// loss = sum m (out - t)^2 / sum m;  gout = 2 m (out - t) / sum m
__global__ void k_loss(const float *out, const float *target, const float *mask, const double *msum,
                       float *gout, double *part, long long P) {
    double acc[1] = {0.0};
    const double inv = *msum > 0.0 ? 1.0 / *msum : 0.0;
    const long long p0 = (long long)blockIdx.x * kRedPx;
    for (long long p = p0 + threadIdx.x; p < p0 + kRedPx && p < P; p += blockDim.x) {
        const double d = (double)out[p] - (double)target[p];
        acc[0] += (double)mask[p] * d * d;
        gout[p] = (float)(2.0 * mask[p] * d * inv);
    }
    acc[0] *= inv;
    block_sum_store<1>(acc, part + blockIdx.x);
}

void launch_loss(const float *out, const float *target, const float *mask, const double *msum,
                 float *gout, double *part, long long P, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(loss_blocks(P)), dim3(256), 0, s, out, target, mask, msum, gout, part, P);
}

__global__ void k_sum_parts(const double *part, int n, double *dst) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += part[k];
    *dst = s;
}

void launch_sum_parts(const double *part, int n, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(64), 0, s, part, n, dst);
}

// ---- parameters -------------------------------------------------------------------
// wf[co][t][ci] (ci < Cin_pad) for the forward; wd[ci][t][co] (co < Cout_pad)
// = w[co][8 - t][ci] for the input gradient (taps flipped, channels swapped).
__global__ void k_wprep(const float *w, int Cin, int Cout, uint16_t *wf, uint16_t *wd) {
    const int Cip = pad32(Cin), Cop = pad32(Cout);
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nf = (long long)Cout * 9 * Cip;
    if (idx < nf) {
        const int ci = (int)(idx % Cip);
        const long long row = idx / Cip;
        wf[idx] = (uint16_t)(ci < Cin ? f2bf(w[row * Cin + ci]) : 0u);
    } else if (idx < nf + (long long)Cin * 9 * Cop) {
        const long long k = idx - nf;
        const int co = (int)(k % Cop);
        const long long row = k / Cop;               // ci * 9 + t
        const int t = (int)(row % 9), ci = (int)(row / 9);
        wd[k] = (uint16_t)(co < Cout ? f2bf(w[((long long)co * 9 + 8 - t) * Cin + ci]) : 0u);
    }
}

void launch_wprep(const float *w, int Cin, int Cout, uint16_t *wf, uint16_t *wd, hipStream_t s) {
    const long long n = (long long)Cout * 9 * pad32(Cin) + (long long)Cin * 9 * pad32(Cout);
    hipLaunchKernelGGL(k_wprep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, Cin, Cout, wf, wd);
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void launch_adam(float *p, const float *g, float *m, float *v, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr,
                       b1, b2, eps, c1, c2);
}

// ---- Poisson problem <-> network tensors -----------------------------------------
// Pixel (h, w) is node (h, w) of the NX x NY node grid (h < H <= NX, w < W <= NY).
// Input channels: source term on free nodes * s_rho; free-node indicator;
// Dirichlet value * s_v on conductor nodes.  Target: phi / s_phi; mask: free.
__global__ void k_snapshot(const double *b, const double *phi, const uint8_t *nc, int NX, int NY,
                           int H, int W, float s_rho, float s_v, float s_phi, uint16_t *x,
                           float *target, float *mask) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (long long)H * W) return;
    const int h = (int)(p / W), w = (int)(p % W);
    const long long node = (long long)h * NY + w;
    const bool freen = nc[node] == 0;
    const double bv = b[node];
    x[3 * p + 0] = (uint16_t)(freen ? f2bf((float)(bv * s_rho)) : 0u);
    x[3 * p + 1] = (uint16_t)(freen ? 0x3F80u : 0u);
    x[3 * p + 2] = (uint16_t)(freen ? 0u : f2bf((float)(bv * s_v)));
    if (phi) {
        target[p] = (float)(phi[node] / s_phi);
        mask[p] = freen ? 1.f : 0.f;
    }
}

void launch_snapshot(const double *b, const double *phi, const uint8_t *node_cond, int NX, int NY,
                     int H, int W, float s_rho, float s_v, float s_phi, uint16_t *x, float *target,
                     float *mask, hipStream_t s) {
    const long long n = (long long)H * W;
    hipLaunchKernelGGL(k_snapshot, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, b, phi, node_cond,
                       NX, NY, H, W, s_rho, s_v, s_phi, x, target, mask);
}

__global__ void k_guess(const float *out, const double *b, const uint8_t *nc, int NX, int NY, int H,
                        int W, float s_phi, double *guess) {
    const long long node = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= (long long)NX * NY) return;
    const int i = (int)(node / NY), j = (int)(node % NY);
    double v = 0.0;
    if (nc[node] != 0) v = b[node];
    else if (i < H && j < W) v = (double)out[(long long)i * W + j] * (double)s_phi;
    guess[node] = v;
}

void launch_guess(const float *out, const double *b, const uint8_t *node_cond, int NX, int NY,
                  int H, int W, float s_phi, double *guess, hipStream_t s) {
    const long long n = (long long)NX * NY;
    hipLaunchKernelGGL(k_guess, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, b, node_cond, NX,
                       NY, H, W, s_phi, guess);
}

// ---- residual learning: samples, stored-sample loads and the corrected start --------
// The start is the linear extrapolation phi_s = 2 phi_1 - phi_2 (phi_1 when
// phi_2 is null); r = b - A phi_s on free nodes with A = 4 - (free
// neighbours), neighbours wrapping on periodic axes (a free node never lies
// on a bounded edge).  Input x [H][W][3] = (bf16(r s_r) on free nodes, free
// indicator, bf16(b s_v) on Dirichlet nodes); target t [H][W] =
// bf16((phi_t - phi_s) s_d) on free nodes.  part (may be null): per-block
// sums of r^2, (phi_t - phi_s)^2 and the free-node count, summed in block
// order by k_rsample_sum into stats.
__device__ __forceinline__ double start_at(const double *p1, const double *p2, long long n) {
    return p2 ? 2.0 * p1[n] - p2[n] : p1[n];
}

constexpr int kRsBlock = 256;

__global__ __launch_bounds__(kRsBlock) void k_rsample(const double *b, const double *p1, const double *p2,
                                                      const double *pt, const uint8_t *nc, int NX, int NY,
                                                      int px, int py, int H, int W, float s_r, float s_v,
                                                      float s_d, uint16_t *x, uint16_t *t, double *part) {
    const long long p = (long long)blockIdx.x * kRsBlock + threadIdx.x;
    double rr = 0.0, dd = 0.0, cnt = 0.0;
    if (p < (long long)H * W) {
        const int i = (int)(p / W), j = (int)(p % W);
        const long long n = (long long)i * NY + j;
        const bool freen = nc[n] == 0;
        uint16_t x0 = 0, x2 = 0, t0 = 0;
        if (freen) {
            double s = 4.0 * start_at(p1, p2, n);
            const int im = i - 1 < 0 ? (px ? NX - 1 : -1) : i - 1;
            const int ip = i + 1 >= NX ? (px ? 0 : -1) : i + 1;
            const int jm = j - 1 < 0 ? (py ? NY - 1 : -1) : j - 1;
            const int jp = j + 1 >= NY ? (py ? 0 : -1) : j + 1;
            long long q;
            if (im >= 0 && !nc[q = (long long)im * NY + j]) s -= start_at(p1, p2, q);
            if (ip >= 0 && !nc[q = (long long)ip * NY + j]) s -= start_at(p1, p2, q);
            if (jm >= 0 && !nc[q = (long long)i * NY + jm]) s -= start_at(p1, p2, q);
            if (jp >= 0 && !nc[q = (long long)i * NY + jp]) s -= start_at(p1, p2, q);
            const double r = b[n] - s;
            x0 = (uint16_t)f2bf((float)(r * s_r));
            rr = r * r;
            cnt = 1.0;
            if (pt) {
                const double d = pt[n] - start_at(p1, p2, n);
                t0 = (uint16_t)f2bf((float)(d * s_d));
                dd = d * d;
            }
        } else {
            x2 = (uint16_t)f2bf((float)(b[n] * s_v));
        }
        x[3 * p + 0] = x0;
        x[3 * p + 1] = (uint16_t)(freen ? 0x3F80u : 0u);
        x[3 * p + 2] = x2;
        if (t) t[p] = t0;
    }
    if (part) {
        double v[3] = {rr, dd, cnt};
        __shared__ double sh[3][kRsBlock];
#pragma unroll
        for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] = v[k];
        __syncthreads();
        for (int off = kRsBlock / 2; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off)
#pragma unroll
                for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 3; ++k) part[3 * (long long)blockIdx.x + k] = sh[k][0];
    }
}

// stats[k] += the sum of the nblk partials of quantity k, in block order
// (one wavefront: lane l sums blocks l, l + 64, ...; the 64 lane sums are
// then added in lane order by lane 0).
__global__ void k_rsample_sum(const double *part, int nblk, double *stats) {
    __shared__ double sh[3][64];
    const int l = threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = l; b < nblk; b += 64)
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k] += part[3 * (long long)b + k];
#pragma unroll
    for (int k = 0; k < 3; ++k) sh[k][l] = s[k];
    __syncthreads();
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double a = 0.0;
            for (int q = 0; q < 64; ++q) a += sh[k][q];
            stats[k] += a;
        }
    }
}

long long rsample_blocks(int H, int W) { return ((long long)H * W + kRsBlock - 1) / kRsBlock; }

void launch_rsample(const double *b, const double *p1, const double *p2, const double *pt,
                    const uint8_t *nc, int NX, int NY, int px, int py, int H, int W, float s_r, float s_v,
                    float s_d, uint16_t *x, uint16_t *t, double *stats, double *part, hipStream_t s) {
    const long long nb = rsample_blocks(H, W);
    hipLaunchKernelGGL(k_rsample, dim3((unsigned)nb), dim3(kRsBlock), 0, s, b, p1, p2, pt, nc, NX, NY, px, py,
                       H, W, s_r, s_v, s_d, x, t, stats ? part : nullptr);
    if (stats) hipLaunchKernelGGL(k_rsample_sum, dim3(1), dim3(64), 0, s, part, (int)nb, stats);
}

// ---- the residual sample without a caller work array ------------------------
// Its per-block partial sums live in `scratch`, a file-scope device array that
// every call on a device shares (each device holds its own copy until the
// process ends).  Host code never passes the array's name to a kernel: the
// device address comes from hipGetSymbolAddress, looked up once per device
// with that device current.  Every block writes its three partials before
// they are summed, so nothing needs clearing between calls; calls that
// overlap on one device race on the array.
constexpr long long kScratchBlocks = 16384;                 // 4,194,304 pixels of 256-pixel blocks
static __device__ __align__(256) double scratch[3 * kScratchBlocks];   // 384 KiB

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double *g_scratch_ptr[kMaxDevices] = {};
}

long long rsample_static_max_pixels() { return kScratchBlocks * kRsBlock; }

hipError_t launch_rsample_static(const double *b, const double *p1, const double *p2, const double *pt,
                                 const uint8_t *nc, int NX, int NY, int px, int py, int H, int W, float s_r,
                                 float s_v, float s_d, uint16_t *x, uint16_t *t, double *stats, hipStream_t s) {
    double *part = nullptr;
    if (stats) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (s) {
            hipDevice_t sd = 0;
            if ((e = hipStreamGetDevice(s, &sd)) != hipSuccess) return e;
            if (sd != dev) return hipErrorInvalidDevice;      // the lookup needs the stream's device current
        }
        if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess) return e;
            g_scratch_ptr[dev] = static_cast<double *>(ptr);
        }
        part = g_scratch_ptr[dev];
    }
    launch_rsample(b, p1, p2, pt, nc, NX, NY, px, py, H, W, s_r, s_v, s_d, x, t, stats, part, s);
    return hipGetLastError();
}

// A stored sample into a batch slot: the input as it is; with t, the target
// (bfloat16 -> float32) and the loss mask (the free-node channel).
__global__ void k_load(const uint16_t *xs, const uint16_t *ts, long long P, uint16_t *x, float *target,
                       float *mask) {
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    x[3 * p + 0] = xs[3 * p + 0];
    x[3 * p + 1] = xs[3 * p + 1];
    x[3 * p + 2] = xs[3 * p + 2];
    if (ts) {
        target[p] = bf2f(ts[p]);
        mask[p] = xs[3 * p + 1] ? 1.f : 0.f;
    }
}

void launch_load(const uint16_t *xs, const uint16_t *ts, long long P, uint16_t *x, float *target, float *mask,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_load, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, xs, ts, P, x, target, mask);
}

// guess = phi_s + out / s_d on free nodes of the window (use_out), phi_s elsewhere.
__global__ void k_rguess(const float *out, const double *p1, const double *p2, const uint8_t *nc, int NX,
                         int NY, int H, int W, float s_d, int use_out, double *guess) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (long long)NX * NY) return;
    const int i = (int)(n / NY), j = (int)(n % NY);
    double v = start_at(p1, p2, n);
    if (use_out && nc[n] == 0 && i < H && j < W) v += (double)out[(long long)i * W + j] / (double)s_d;
    guess[n] = v;
}

void launch_rguess(const float *out, const double *p1, const double *p2, const uint8_t *nc, int NX, int NY,
                   int H, int W, float s_d, int use_out, double *guess, hipStream_t s) {
    const long long n = (long long)NX * NY;
    hipLaunchKernelGGL(k_rguess, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, p1, p2, nc, NX, NY,
                       H, W, s_d, use_out, guess);
}

// ---- time extrapolation of the potential ------------------------------------
// out = coef[0] phi[0] + coef[1] phi[1] + ... (added in this order).
__global__ void k_extrapolate_k(ExtrapArgs a) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    double s = a.c[0] * a.p[0][i];
    for (int k = 1; k < a.K; ++k) s = s + a.c[k] * a.p[k][i];
    a.out[i] = s;
}

void launch_extrapolate(const ExtrapArgs &a, hipStream_t s) {
    if (a.n <= 0) return;
    hipLaunchKernelGGL(k_extrapolate_k, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
}

// ---- coarse residual learning -----------------------------------------------
// Pixel (h, w) of the network stands for the f x f block of nodes
// (h f + p, w f + q), p, q < f (f divides 16), so the network's receptive
// field spans the whole grid.  Input x [H][W][3] = (bf16(R/f^2 s_r),
// bf16(F/f^2), bf16(V/f^2 s_v)) and target t [H][W] = bf16(D/f^2 s_d), with
// R, D, F the sums over the block's free nodes of the residual r of the
// extrapolated start, of (phi_t - phi_s) and of 1, and V the sum of the
// Dirichlet values of its conductor nodes; every sum adds the block's nodes
// in row-major order (p outer, q inner), starting from 0.  One block of 256
// threads covers a 16 x 16 tile of nodes: each thread computes one node's
// terms into LDS, then one thread per pixel of the tile adds its block.
// part (may be null): per-block sums, in pixel order, of (R/f^2)^2,
// (D/f^2)^2 and the count of pixels with a free node.
constexpr int kCsTile = 16;

__global__ __launch_bounds__(256) void k_csample(const double *b, const double *p1, const double *p2,
                                                 const double *pt, const uint8_t *nc, int NX, int NY, int px,
                                                 int py, int f, int H, int W, float s_r, float s_v, float s_d,
                                                 uint16_t *x, uint16_t *t, double *part) {
    __shared__ double sr[kCsTile * kCsTile], sv[kCsTile * kCsTile], sd[kCsTile * kCsTile];
    __shared__ unsigned char sf[kCsTile * kCsTile];
    __shared__ double st[3][kCsTile * kCsTile];
    const int tid = threadIdx.x;
    const int tiles_w = (W * f + kCsTile - 1) / kCsTile;
    const int bi = blockIdx.x / tiles_w, bj = blockIdx.x % tiles_w;
    const int i = bi * kCsTile + tid / kCsTile, j = bj * kCsTile + tid % kCsTile;
    double r = 0.0, v = 0.0, d = 0.0;
    unsigned char fr = 0;
    if (i < H * f && j < W * f) {
        const long long n = (long long)i * NY + j;
        if (nc[n] == 0) {
            double s = 4.0 * start_at(p1, p2, n);
            const int im = i - 1 < 0 ? (px ? NX - 1 : -1) : i - 1;
            const int ip = i + 1 >= NX ? (px ? 0 : -1) : i + 1;
            const int jm = j - 1 < 0 ? (py ? NY - 1 : -1) : j - 1;
            const int jp = j + 1 >= NY ? (py ? 0 : -1) : j + 1;
            long long q;
            if (im >= 0 && !nc[q = (long long)im * NY + j]) s -= start_at(p1, p2, q);
            if (ip >= 0 && !nc[q = (long long)ip * NY + j]) s -= start_at(p1, p2, q);
            if (jm >= 0 && !nc[q = (long long)i * NY + jm]) s -= start_at(p1, p2, q);
            if (jp >= 0 && !nc[q = (long long)i * NY + jp]) s -= start_at(p1, p2, q);
            r = b[n] - s;
            if (pt) d = pt[n] - start_at(p1, p2, n);
            fr = 1;
        } else {
            v = b[n];
        }
    }
    sr[tid] = r;
    sv[tid] = v;
    sd[tid] = d;
    sf[tid] = fr;
    __syncthreads();
    const int per = kCsTile / f;                 // pixels per tile edge
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    if (tid < per * per) {
        const int a = tid / per, c = tid % per;
        const int h = bi * per + a, w = bj * per + c;
        if (h < H && w < W) {
            double R = 0.0, V = 0.0, D = 0.0, F = 0.0;
            for (int pp = 0; pp < f; ++pp)
                for (int qq = 0; qq < f; ++qq) {
                    const int l = (a * f + pp) * kCsTile + (c * f + qq);
                    if (sf[l]) {
                        R += sr[l];
                        D += sd[l];
                        F += 1.0;
                    } else {
                        V += sv[l];
                    }
                }
            const double inv = 1.0 / (double)(f * f);
            const long long p = (long long)h * W + w;
            const double rm = R * inv, dm = D * inv;
            x[3 * p + 0] = (uint16_t)f2bf((float)(rm * (double)s_r));
            x[3 * p + 1] = (uint16_t)f2bf((float)(F * inv));
            x[3 * p + 2] = (uint16_t)f2bf((float)(V * inv * (double)s_v));
            if (t) t[p] = (uint16_t)f2bf((float)(dm * (double)s_d));
            q0 = rm * rm;
            q1 = dm * dm;
            q2 = F > 0.0 ? 1.0 : 0.0;
        }
    }
    if (part) {
        st[0][tid] = q0;
        st[1][tid] = q1;
        st[2][tid] = q2;
        __syncthreads();
        if (tid == 0) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0;
            for (int k = 0; k < per * per; ++k) {
                a0 += st[0][k];
                a1 += st[1][k];
                a2 += st[2][k];
            }
            part[3 * (long long)blockIdx.x + 0] = a0;
            part[3 * (long long)blockIdx.x + 1] = a1;
            part[3 * (long long)blockIdx.x + 2] = a2;
        }
    }
}

long long csample_blocks(int f, int H, int W) {
    return (long long)((H * f + kCsTile - 1) / kCsTile) * ((W * f + kCsTile - 1) / kCsTile);
}

void launch_csample(const double *b, const double *p1, const double *p2, const double *pt, const uint8_t *nc,
                    int NX, int NY, int px, int py, int f, int H, int W, float s_r, float s_v, float s_d,
                    uint16_t *x, uint16_t *t, double *stats, double *part, hipStream_t s) {
    const long long nb = csample_blocks(f, H, W);
    hipLaunchKernelGGL(k_csample, dim3((unsigned)nb), dim3(kCsTile * kCsTile), 0, s, b, p1, p2, pt, nc, NX, NY,
                       px, py, f, H, W, s_r, s_v, s_d, x, t, stats ? part : nullptr);
    if (stats) hipLaunchKernelGGL(k_rsample_sum, dim3(1), dim3(64), 0, s, part, (int)nb, stats);
}

// Lower and upper pixel of node index i on an axis of n pixels of f nodes and
// the upper pixel's weight: the node lies at pixel coordinate (i + 1/2)/f - 1/2
// (pixel centres at integers); beyond [0, n - 1] the index wraps (wrap) or is
// clamped to the edge pixel.
__device__ __forceinline__ void axis_weights(int i, int f, int n, bool wrap, int &lo, int &hi, double &a) {
    const double u = ((double)i + 0.5) / (double)f - 0.5;
    const double fl = floor(u);
    a = u - fl;
    lo = (int)fl;
    hi = lo + 1;
    if (wrap) {
        lo = lo < 0 ? lo + n : lo;
        hi = hi >= n ? hi - n : hi;
    } else {
        lo = min(max(lo, 0), n - 1);
        hi = min(max(hi, 0), n - 1);
    }
}

// guess = phi_s + c / s_d on the free nodes of the covered H f x W f region
// (use_out), c the bilinear interpolation of the coarse output, weights
// (1-a)(1-b), a(1-b), (1-a)b, ab added in that order; phi_s elsewhere.  An
// axis wraps when it is periodic and covered exactly.
__global__ void k_cguess(const float *out, const double *p1, const double *p2, const uint8_t *nc, int NX,
                         int NY, int px, int py, int f, int H, int W, float s_d, int use_out, double *guess) {
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (long long)NX * NY) return;
    const int i = (int)(n / NY), j = (int)(n % NY);
    double v = start_at(p1, p2, n);
    if (use_out && nc[n] == 0 && i < H * f && j < W * f) {
        int h0, h1, w0, w1;
        double a, bq;
        axis_weights(i, f, H, px && H * f == NX, h0, h1, a);
        axis_weights(j, f, W, py && W * f == NY, w0, w1, bq);
        double c = (1.0 - a) * (1.0 - bq) * (double)out[(long long)h0 * W + w0];
        c = c + a * (1.0 - bq) * (double)out[(long long)h1 * W + w0];
        c = c + (1.0 - a) * bq * (double)out[(long long)h0 * W + w1];
        c = c + a * bq * (double)out[(long long)h1 * W + w1];
        v = v + c / (double)s_d;
    }
    guess[n] = v;
}

void launch_cguess(const float *out, const double *p1, const double *p2, const uint8_t *nc, int NX, int NY,
                   int px, int py, int f, int H, int W, float s_d, int use_out, double *guess, hipStream_t s) {
    const long long n = (long long)NX * NY;
    hipLaunchKernelGGL(k_cguess, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, p1, p2, nc, NX, NY, px,
                       py, f, H, W, s_d, use_out, guess);
}

} // namespace unet
