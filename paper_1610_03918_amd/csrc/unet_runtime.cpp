// Host runtime of the learned warm start (C ABI of pic_unet.h): layer table,
// workspace carving, and the order of the forward / backward launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/pic_unet.h"
#include "ctx_view.h"
#include "unet_internal.h"

using namespace unet;

namespace {

struct Layer {
    int cin, cout, level;
    long long w_off, b_off;
    // inputs: full-resolution source and optional half-resolution source (upsampled)
    int src_act, up_act;         // activation index, -1 = network input / none, -2 = pooled of level
};

// Network order: encoder level 0..3 (two convolutions each, the first of
// levels 1..3 reading the pooled output of the level above), then decoder
// levels 2, 1, 0 (the first reading [upsampled deeper output, skip]).
struct Net {
    Layer L[kNConv];
    long long head_off = 0, count = 0;
    Net()
    {
        const int ch[kLevels] = {16, 32, 64, 128};
        long long off = 0;
        int k = 0;
        int cin = kInCh;
        for (int l = 0; l < kLevels; l++) {
            for (int r = 0; r < 2; r++) {
                Layer &y = L[k];
                y.cin = r == 0 ? cin : ch[l];
                y.cout = ch[l];
                y.level = l;
                y.up_act = -1;
                y.src_act = r == 1 ? k - 1 : (l == 0 ? -1 : -2);
                k++;
            }
            cin = ch[l];
        }
        for (int l = kLevels - 2; l >= 0; l--) {
            for (int r = 0; r < 2; r++) {
                Layer &y = L[k];
                y.cin = r == 0 ? cin + ch[l] : ch[l];
                y.cout = ch[l];
                y.level = l;
                y.up_act = r == 0 ? k - 1 : -1;
                y.src_act = r == 0 ? 2 * l + 1 : k - 1;   // skip: second encoder conv of level l
                k++;
            }
            cin = ch[l];
        }
        for (int q = 0; q < kNConv; q++) {
            L[q].w_off = off;
            off += (long long)L[q].cout * 9 * L[q].cin;
            L[q].b_off = off;
            off += L[q].cout;
        }
        head_off = off;
        count = off + 17;
    }
};

const Net &net()
{
    static Net n;
    return n;
}

struct Carve {
    size_t off = 0;
    char *base = nullptr;
    template <class T> T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

constexpr long long kPartFloats = 8ll << 20;   // cap of the weight-gradient partial sums

} // namespace

struct pic_unet {
    int B = 0, H = 0, W = 0;
    long long P0 = 0;
    hipStream_t stream = nullptr;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *wf[kNConv] = {}, *wd[kNConv] = {};
    uint16_t *x = nullptr;
    uint16_t *act[kNConv] = {};
    uint16_t *pooled[kLevels] = {};
    float *out = nullptr, *target = nullptr, *mask = nullptr, *gout = nullptr;
    float *G[kLevels - 1] = {};
    float *g1 = nullptr, *gp = nullptr;
    uint16_t *gy = nullptr;
    float *part = nullptr, *bpart = nullptr;
    double *dpart = nullptr, *scal = nullptr;   // scal[0] mask sum, scal[1] loss
    int ndpart = 0;
    int adam_t = 0;
    int pw = 0;                                  // circular padding along W
    bool dirty = true;
    bool timing = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double timed_ms = 0.0;
    int timed_n = 0;
    std::string err;
};

namespace {

pic_status ufail(pic_unet *u, pic_status st, const std::string &msg)
{
    if (u) u->err = msg;
    return st;
}

#define UCHK(u, call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ufail(u, PIC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int chan(int level) { return 16 << level; }

// Lays out every buffer of a network over B x H x W; base == nullptr only measures.
size_t carve(pic_unet *u, char *base, int B, int H, int W)
{
    const Net &N = net();
    Carve cv;
    cv.base = base;
    const long long P0 = (long long)B * H * W;
    auto P = [&](int l) { return (long long)B * (H >> l) * (W >> l); };
    uint16_t *wf[kNConv], *wd[kNConv], *act[kNConv], *pooled[kLevels] = {};
    for (int k = 0; k < kNConv; k++) {
        wf[k] = cv.take<uint16_t>((size_t)N.L[k].cout * 9 * pad32(N.L[k].cin));
        wd[k] = cv.take<uint16_t>((size_t)N.L[k].cin * 9 * pad32(N.L[k].cout));
    }
    uint16_t *x = cv.take<uint16_t>((size_t)P0 * kInCh);
    for (int k = 0; k < kNConv; k++) act[k] = cv.take<uint16_t>((size_t)P(N.L[k].level) * N.L[k].cout);
    for (int l = 1; l < kLevels; l++) pooled[l] = cv.take<uint16_t>((size_t)P(l) * chan(l - 1));
    float *out = cv.take<float>(P0), *target = cv.take<float>(P0), *mask = cv.take<float>(P0);
    float *gout = cv.take<float>(P0);
    float *G[kLevels - 1];
    for (int l = 0; l < kLevels - 1; l++) G[l] = cv.take<float>((size_t)P(l) * (chan(l) + chan(l + 1)));
    float *g1 = cv.take<float>((size_t)P0 * 16);
    float *gp = cv.take<float>((size_t)P0 * 4);
    uint16_t *gy = cv.take<uint16_t>((size_t)P0 * 16);
    float *part = cv.take<float>((size_t)kPartFloats);
    float *bpart = cv.take<float>((size_t)1024 * 128);
    const int nd = std::max(17 * head_bwd_blocks(P0), loss_blocks(P0));
    double *dpart = cv.take<double>((size_t)nd);
    double *scal = cv.take<double>(8);
    if (u) {
        for (int k = 0; k < kNConv; k++) {
            u->wf[k] = wf[k];
            u->wd[k] = wd[k];
            u->act[k] = act[k];
        }
        for (int l = 0; l < kLevels; l++) u->pooled[l] = pooled[l];
        for (int l = 0; l < kLevels - 1; l++) u->G[l] = G[l];
        u->x = x;
        u->out = out;
        u->target = target;
        u->mask = mask;
        u->gout = gout;
        u->g1 = g1;
        u->gp = gp;
        u->gy = gy;
        u->part = part;
        u->bpart = bpart;
        u->dpart = dpart;
        u->ndpart = nd;
        u->scal = scal;
    }
    return cv.off + 256;
}

// Full- and half-resolution inputs of convolution k.
void conv_inputs(const pic_unet *u, int k, const uint16_t **src, int *Cs, const uint16_t **up, int *Cu)
{
    const Layer &y = net().L[k];
    *up = nullptr;
    *Cu = 0;
    if (y.up_act >= 0) {
        *up = u->act[y.up_act];
        *Cu = net().L[y.up_act].cout;
    }
    if (y.src_act == -1) {
        *src = u->x;
        *Cs = kInCh;
    } else if (y.src_act == -2) {
        *src = u->pooled[y.level];
        *Cs = chan(y.level - 1);
    } else {
        *src = u->act[y.src_act];
        *Cs = net().L[y.src_act].cout;
    }
}

void enqueue_forward(pic_unet *u)
{
    const Net &N = net();
    hipStream_t s = u->stream;
    if (u->dirty) {
        for (int k = 0; k < kNConv; k++)
            launch_wprep(u->params + N.L[k].w_off, N.L[k].cin, N.L[k].cout, u->wf[k], u->wd[k], s);
        u->dirty = false;
    }
    for (int k = 0; k < kNConv; k++) {
        const Layer &y = N.L[k];
        const int l = y.level;
        if (y.src_act == -2)
            launch_pool(u->act[2 * l - 1], u->pooled[l], u->B, u->H >> (l - 1), u->W >> (l - 1), chan(l - 1), s);
        ConvArgs a{};
        a.B = u->B;
        a.H = u->H >> l;
        a.W = u->W >> l;
        conv_inputs(u, k, &a.src, &a.Cs, &a.up, &a.Cu);
        a.Cin_pad = pad32(y.cin);
        a.wt = u->wf[k];
        a.bias = u->params + y.b_off;
        a.Cout = y.cout;
        a.out = u->act[k];
        a.pw = u->pw;
        launch_conv(a, false, s);
    }
    launch_head_fwd(u->act[kNConv - 1], u->params + N.head_off, u->out, u->P0, s);
}

// Weight gradient and (unless k == 0) input gradient of convolution k from u->gy.
void conv_backward(pic_unet *u, int k, float *gx)
{
    const Net &N = net();
    const Layer &y = N.L[k];
    hipStream_t s = u->stream;
    const int l = y.level, H = u->H >> l, W = u->W >> l;
    WgradArgs w{};
    w.B = u->B;
    w.H = H;
    w.W = W;
    w.gy = u->gy;
    w.Cout = y.cout;
    conv_inputs(u, k, &w.src, &w.Cs, &w.up, &w.Cu);
    w.Cin_pad = pad32(y.cin);
    const int chunks = w.Cin_pad / kKChunk;
    const int per_split = (y.cout % 32 == 0 ? y.cout / 32 : y.cout / 16) * chunks;
    const long long per_part = (long long)y.cout * 9 * w.Cin_pad;
    // about four pixel tiles per block, at least ~1024 blocks where the image allows
    const int tiles = wgrad_tiles(u->B, H, W);
    int ns = std::max((tiles + 3) / 4, (1024 + per_split - 1) / per_split);
    ns = std::min(ns, tiles);
    ns = (int)std::min<long long>(ns, std::max(1ll, kPartFloats / per_part));
    ns = std::min(ns, 1024);
    w.nsplit = ns;
    w.part = u->part;
    w.bpart = u->bpart;
    w.pw = u->pw;
    launch_wgrad(w, chunks, s);
    launch_wgrad_reduce(u->part, u->bpart, ns, y.cout, y.cin, w.Cin_pad, u->grads + y.w_off,
                        u->grads + y.b_off, s);
    if (!gx) return;
    ConvArgs a{};
    a.B = u->B;
    a.H = H;
    a.W = W;
    a.src = u->gy;
    a.Cs = y.cout;
    a.up = nullptr;
    a.Cu = 0;
    a.Cin_pad = pad32(y.cout);
    a.wt = u->wd[k];
    a.bias = nullptr;
    a.Cout = y.cin;
    a.out = gx;
    a.pw = u->pw;
    launch_conv(a, true, s);
}

void relu_bwd(pic_unet *u, int level, int C, const float *ga, int sa, int oa, int a_up, const float *gb,
              const uint16_t *h)
{
    ReluBwdArgs r{};
    r.B = u->B;
    r.H = u->H >> level;
    r.W = u->W >> level;
    r.C = C;
    r.ga = ga;
    r.sa = sa;
    r.oa = oa;
    r.a_up = a_up;
    r.gb = gb;
    r.h = h;
    r.gy = u->gy;
    launch_relu_bwd(r, u->stream);
}

void enqueue_backward(pic_unet *u)
{
    const Net &N = net();
    hipStream_t s = u->stream;
    const int nb = head_bwd_blocks(u->P0);
    launch_head_bwd(u->act[13], u->params + N.head_off, u->gout, u->gy, u->dpart, u->P0, s);
    launch_head_finalize(u->dpart, nb, u->grads + N.head_off, s);
    // decoder, finest level first: convs 13,12 (level 0), 11,10 (level 1), 9,8 (level 2)
    for (int l = 0; l < kLevels - 1; l++) {
        const int kb = 13 - 2 * l, ka = kb - 1;
        const int C = chan(l), Cin = C + chan(l + 1);
        conv_backward(u, kb, u->g1);
        relu_bwd(u, l, C, u->g1, C, 0, 0, nullptr, u->act[ka]);
        conv_backward(u, ka, u->G[l]);
        // gradient of the deeper output feeding the upsampling (conv ka - 1)
        relu_bwd(u, l + 1, chan(l + 1), u->G[l], Cin, 0, 1, nullptr, u->act[ka - 1]);
    }
    // encoder, deepest level first: convs 7,6 (level 3), 5,4 (2), 3,2 (1), 1,0 (0)
    for (int l = kLevels - 1; l >= 0; l--) {
        const int kb = 2 * l + 1, ka = 2 * l;
        const int C = chan(l);
        if (l < kLevels - 1) {
            // skip part of the decoder's input gradient plus the pooling adjoint
            relu_bwd(u, l, C, u->G[l], C + chan(l + 1), chan(l + 1), 0, u->gp, u->act[kb]);
        }
        conv_backward(u, kb, u->g1);
        relu_bwd(u, l, C, u->g1, C, 0, 0, nullptr, u->act[ka]);
        conv_backward(u, ka, l > 0 ? u->gp : nullptr);
    }
}

} // namespace

extern "C" {

int64_t pic_unet_param_count(void) { return net().count; }

pic_status pic_unet_layer_info(int32_t k, pic_unet_layer *out)
{
    if (!out || k < 0 || k > kNConv) return PIC_ERR_ARG;
    const Net &N = net();
    if (k == kNConv) {
        *out = pic_unet_layer{16, 1, 0, 0, N.head_off, N.head_off + 16};
        return PIC_OK;
    }
    const Layer &y = N.L[k];
    *out = pic_unet_layer{y.cin, y.cout, y.level, 0, y.w_off, y.b_off};
    return PIC_OK;
}

static bool shape_ok(int B, int H, int W)
{
    return B >= 1 && B <= 64 && H >= 8 && W >= 8 && H % 8 == 0 && W % 8 == 0 && H <= 8192 && W <= 8192;
}

pic_status pic_unet_workspace_size(int32_t batch, int32_t H, int32_t W, size_t *bytes)
{
    if (!bytes || !shape_ok(batch, H, W)) return PIC_ERR_ARG;
    *bytes = carve(nullptr, nullptr, batch, H, W);
    return PIC_OK;
}

pic_status pic_unet_create(int32_t batch, int32_t H, int32_t W, float *params, float *grads,
                           float *adam_m, float *adam_v, void *workspace, size_t workspace_bytes,
                           void *stream, pic_unet **out)
{
    if (!out) return PIC_ERR_ARG;
    *out = nullptr;
    if (!shape_ok(batch, H, W) || !params || !grads || !adam_m || !adam_v || !workspace) return PIC_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return PIC_ERR_ARG;
    if (workspace_bytes < carve(nullptr, nullptr, batch, H, W)) return PIC_ERR_ARG;
    pic_unet *u = new pic_unet();
    u->B = batch;
    u->H = H;
    u->W = W;
    u->P0 = (long long)batch * H * W;
    u->stream = static_cast<hipStream_t>(stream);
    u->params = params;
    u->grads = grads;
    u->m = adam_m;
    u->v = adam_v;
    carve(u, static_cast<char *>(workspace), batch, H, W);
    *out = u;
    return PIC_OK;
}

pic_status pic_unet_io_buffers(pic_unet *u, pic_unet_io *io)
{
    if (!u || !io) return PIC_ERR_ARG;
    *io = pic_unet_io{u->x, u->out, u->target, u->mask, u->gout};
    return PIC_OK;
}

pic_status pic_unet_params_changed(pic_unet *u)
{
    if (!u) return PIC_ERR_ARG;
    u->dirty = true;
    return PIC_OK;
}

pic_status pic_unet_forward(pic_unet *u)
{
    if (!u) return PIC_ERR_ARG;
    if (u->timing) UCHK(u, hipEventRecord(u->e0, u->stream));
    enqueue_forward(u);
    if (u->timing) {
        UCHK(u, hipEventRecord(u->e1, u->stream));
        UCHK(u, hipEventSynchronize(u->e1));
        float ms = 0.f;
        UCHK(u, hipEventElapsedTime(&ms, u->e0, u->e1));
        u->timed_ms += ms;
        u->timed_n++;
    }
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

pic_status pic_unet_loss(pic_unet *u, double *loss)
{
    if (!u) return PIC_ERR_ARG;
    const int nb = loss_blocks(u->P0);
    launch_mask_sum(u->mask, u->dpart, u->P0, u->stream);
    launch_sum_parts(u->dpart, nb, u->scal, u->stream);
    launch_loss(u->out, u->target, u->mask, u->scal, u->gout, u->dpart, u->P0, u->stream);
    launch_sum_parts(u->dpart, nb, u->scal + 1, u->stream);
    UCHK(u, hipGetLastError());
    double h = 0.0;
    UCHK(u, hipMemcpyAsync(&h, u->scal + 1, sizeof(double), hipMemcpyDeviceToHost, u->stream));
    UCHK(u, hipStreamSynchronize(u->stream));
    if (loss) *loss = h;
    return PIC_OK;
}

pic_status pic_unet_backward(pic_unet *u)
{
    if (!u) return PIC_ERR_ARG;
    if (u->dirty) return ufail(u, PIC_ERR_STATE, "pic_unet_backward: no forward pass with the current parameters");
    enqueue_backward(u);
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

pic_status pic_unet_adam(pic_unet *u, float lr, float beta1, float beta2, float eps)
{
    if (!u || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return ufail(u, PIC_ERR_ARG, "pic_unet_adam: bad hyper-parameters");
    u->adam_t++;
    const float c1 = 1.f - (float)std::pow((double)beta1, u->adam_t);
    const float c2 = 1.f - (float)std::pow((double)beta2, u->adam_t);
    launch_adam(u->params, u->grads, u->m, u->v, net().count, lr, beta1, beta2, eps, c1, c2, u->stream);
    u->dirty = true;
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

pic_status pic_unet_snapshot(pic_unet *u, int32_t slot, const double *b, const double *phi,
                             const uint8_t *node_cond, int32_t NX, int32_t NY, float s_rho,
                             float s_v, float s_phi)
{
    if (!u) return PIC_ERR_ARG;
    if (slot < 0 || slot >= u->B || !b || !node_cond || NX < u->H || NY < u->W || (phi && !(s_phi != 0.f)))
        return ufail(u, PIC_ERR_ARG, "pic_unet_snapshot: bad slot, pointer or grid smaller than the network");
    const long long off = (long long)slot * u->H * u->W;
    launch_snapshot(b, phi, node_cond, NX, NY, u->H, u->W, s_rho, s_v, s_phi, u->x + off * kInCh,
                    u->target + off, u->mask + off, u->stream);
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

pic_status pic_unet_guess(pic_unet *u, int32_t slot, const double *b, const uint8_t *node_cond,
                          int32_t NX, int32_t NY, float s_phi, double *guess)
{
    if (!u) return PIC_ERR_ARG;
    if (slot < 0 || slot >= u->B || !b || !node_cond || !guess || NX < u->H || NY < u->W)
        return ufail(u, PIC_ERR_ARG, "pic_unet_guess: bad slot, pointer or grid smaller than the network");
    launch_guess(u->out + (long long)slot * u->H * u->W, b, node_cond, NX, NY, u->H, u->W, s_phi, guess,
                 u->stream);
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

// The network's stream waits for the work queued so far on `other`.
static pic_status after_stream(pic_unet *u, hipStream_t other)
{
    if (other == u->stream) return PIC_OK;
    hipEvent_t ev = nullptr;
    UCHK(u, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    hipError_t e = hipEventRecord(ev, other);
    if (e == hipSuccess) e = hipStreamWaitEvent(u->stream, ev, 0);
    (void)hipEventDestroy(ev);
    UCHK(u, e);
    return PIC_OK;
}

pic_status pic_solve_learned(pic_ctx *ctx, pic_unet *u, const double *b, float s_rho, float s_v,
                             float s_phi, double *guess, pic_solve_info *info)
{
    if (!ctx || !u) return PIC_ERR_ARG;
    const uint8_t *nc = nullptr;
    int32_t NX = 0, NY = 0;
    pic_status st = pic_node_map(ctx, 0, &nc, nullptr, &NX, &NY);
    if (st != PIC_OK) return st;
    PicCtxView v;
    if ((st = pic_ctx_view(ctx, 0, &v)) != PIC_OK) return st;
    // b was assembled on the context's stream
    if ((st = after_stream(u, v.stream)) != PIC_OK) return st;
    if ((st = pic_unet_snapshot(u, 0, b, nullptr, nc, NX, NY, s_rho, s_v, s_phi)) != PIC_OK) return st;
    if ((st = pic_unet_forward(u)) != PIC_OK) return st;
    if ((st = pic_unet_guess(u, 0, b, nc, NX, NY, s_phi, guess)) != PIC_OK) return st;
    UCHK(u, hipStreamSynchronize(u->stream));
    return pic_solve(ctx, 2, guess, info);
}

pic_status pic_unet_set_periodic(pic_unet *u, int32_t periodic_w)
{
    if (!u || (periodic_w != 0 && periodic_w != 1)) return ufail(u, PIC_ERR_ARG, "periodic_w must be 0 or 1");
    u->pw = periodic_w;
    return PIC_OK;
}

pic_status pic_unet_residual_sample_work_bytes(int32_t H, int32_t W, size_t *bytes)
{
    if (!bytes || H < 1 || W < 1) return PIC_ERR_ARG;
    *bytes = (size_t)rsample_blocks(H, W) * 3 * sizeof(double);
    return PIC_OK;
}

pic_status pic_unet_residual_sample(const double *b, const double *phi_1, const double *phi_2,
                                    const double *phi_t, const uint8_t *node_cond, int32_t NX, int32_t NY,
                                    int32_t periodic_x, int32_t periodic_y, int32_t H, int32_t W, float s_r,
                                    float s_v, float s_d, uint16_t *x, uint16_t *t, double *stats,
                                    void *work, size_t work_bytes, void *stream)
{
    if (!b || !phi_1 || !node_cond || !x || H < 1 || W < 1 || H > NX || W > NY || (t && !phi_t)) return PIC_ERR_ARG;
    if (stats && (!work || work_bytes < (size_t)rsample_blocks(H, W) * 3 * sizeof(double))) return PIC_ERR_ARG;
    launch_rsample(b, phi_1, phi_2, phi_t, node_cond, NX, NY, periodic_x ? 1 : 0, periodic_y ? 1 : 0, H, W,
                   s_r, s_v, s_d, x, t, stats, static_cast<double *>(work), static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_ERR_HIP;
}

pic_status pic_unet_residual_sample_noalloc(const double *b, const double *phi_1, const double *phi_2,
                                            const double *phi_t, const uint8_t *node_cond, int32_t NX,
                                            int32_t NY, int32_t periodic_x, int32_t periodic_y, int32_t H,
                                            int32_t W, float s_r, float s_v, float s_d, uint16_t *x, uint16_t *t,
                                            double *stats, void *stream)
{
    if (!b || !phi_1 || !node_cond || !x || H < 1 || W < 1 || H > NX || W > NY || (t && !phi_t)) return PIC_ERR_ARG;
    if (stats && (long long)H * W > rsample_static_max_pixels()) return PIC_ERR_CAPACITY;
    hipError_t e = launch_rsample_static(b, phi_1, phi_2, phi_t, node_cond, NX, NY, periodic_x ? 1 : 0,
                                         periodic_y ? 1 : 0, H, W, s_r, s_v, s_d, x, t, stats,
                                         static_cast<hipStream_t>(stream));
    if (e == hipErrorInvalidDevice) return PIC_ERR_ARG;
    return e == hipSuccess ? PIC_OK : PIC_ERR_HIP;
}

pic_status pic_unet_load(pic_unet *u, int32_t slot, const uint16_t *x, const uint16_t *t)
{
    if (!u) return PIC_ERR_ARG;
    if (slot < 0 || slot >= u->B || !x) return ufail(u, PIC_ERR_ARG, "pic_unet_load: bad slot or null input");
    const long long P = (long long)u->H * u->W, off = (long long)slot * P;
    launch_load(x, t, P, u->x + off * kInCh, u->target + off, u->mask + off, u->stream);
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

pic_status pic_unet_extrapolate(const double *const *phi, const double *coef, int32_t K, int64_t n, double *out,
                                void *stream)
{
    if (!phi || !coef || !out || K < 1 || K > kExtrapMax || n < 0) return PIC_ERR_ARG;
    ExtrapArgs a{};
    for (int k = 0; k < K; ++k) {
        if (!phi[k]) return PIC_ERR_ARG;
        a.p[k] = phi[k];
        a.c[k] = coef[k];
    }
    a.K = K;
    a.n = n;
    a.out = out;
    launch_extrapolate(a, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_ERR_HIP;
}

pic_status pic_unet_residual_guess(pic_unet *u, int32_t slot, const double *phi_1, const double *phi_2,
                                   const uint8_t *node_cond, int32_t NX, int32_t NY, float s_d,
                                   int32_t use_output, double *guess)
{
    if (!u) return PIC_ERR_ARG;
    if (slot < 0 || slot >= u->B || !phi_1 || !node_cond || !guess || NX < u->H || NY < u->W || !(s_d != 0.f))
        return ufail(u, PIC_ERR_ARG, "pic_unet_residual_guess: bad slot, pointer, scale or grid");
    launch_rguess(u->out + (long long)slot * u->H * u->W, phi_1, phi_2, node_cond, NX, NY, u->H, u->W, s_d,
                  use_output ? 1 : 0, guess, u->stream);
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

pic_status pic_solve_learned_residual(pic_ctx *ctx, pic_unet *u, float s_r, float s_v, float s_d,
                                      double *guess, pic_solve_info *info)
{
    if (!ctx || !u) return PIC_ERR_ARG;
    if (u->B < 1) return PIC_ERR_ARG;
    PicCtxView v;
    pic_status st = pic_ctx_view(ctx, 0, &v);
    if (st != PIC_OK) return st;
    if (!guess || v.NX < u->H || v.NY < u->W) return ufail(u, PIC_ERR_ARG, "pic_solve_learned_residual: grid or guess");
    // the right-hand side and the potentials were written on the context's stream
    if ((st = after_stream(u, v.stream)) != PIC_OK) return st;
    launch_rsample(v.b, v.phi, v.phi_prev, nullptr, v.node_cond, v.NX, v.NY, v.px, v.py, u->H, u->W, s_r, s_v,
                   s_d, u->x, nullptr, nullptr, nullptr, u->stream);
    if ((st = pic_unet_forward(u)) != PIC_OK) return st;
    launch_rguess(u->out, v.phi, v.phi_prev, v.node_cond, v.NX, v.NY, u->H, u->W, s_d, 1, guess, u->stream);
    UCHK(u, hipGetLastError());
    UCHK(u, hipStreamSynchronize(u->stream));
    return pic_solve(ctx, 4, guess, info);
}

static bool coarse_factor_ok(int f) { return f == 1 || f == 2 || f == 4 || f == 8 || f == 16; }

pic_status pic_unet_coarse_sample_work_bytes(int32_t f, int32_t H, int32_t W, size_t *bytes)
{
    if (!bytes || !coarse_factor_ok(f) || H < 1 || W < 1) return PIC_ERR_ARG;
    *bytes = (size_t)csample_blocks(f, H, W) * 3 * sizeof(double);
    return PIC_OK;
}

pic_status pic_unet_coarse_sample(const double *b, const double *phi_1, const double *phi_2, const double *phi_t,
                                  const uint8_t *node_cond, int32_t NX, int32_t NY, int32_t periodic_x,
                                  int32_t periodic_y, int32_t f, int32_t H, int32_t W, float s_r, float s_v,
                                  float s_d, uint16_t *x, uint16_t *t, double *stats, void *work,
                                  size_t work_bytes, void *stream)
{
    if (!b || !phi_1 || !node_cond || !x || !coarse_factor_ok(f) || H < 1 || W < 1 || (long long)H * f > NX ||
        (long long)W * f > NY || (t && !phi_t))
        return PIC_ERR_ARG;
    if (stats && (!work || work_bytes < (size_t)csample_blocks(f, H, W) * 3 * sizeof(double))) return PIC_ERR_ARG;
    launch_csample(b, phi_1, phi_2, phi_t, node_cond, NX, NY, periodic_x ? 1 : 0, periodic_y ? 1 : 0, f, H, W, s_r,
                   s_v, s_d, x, t, stats, static_cast<double *>(work), static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_ERR_HIP;
}

pic_status pic_unet_coarse_guess(pic_unet *u, int32_t slot, const double *phi_1, const double *phi_2,
                                 const uint8_t *node_cond, int32_t NX, int32_t NY, int32_t periodic_x,
                                 int32_t periodic_y, int32_t f, float s_d, int32_t use_output, double *guess)
{
    if (!u) return PIC_ERR_ARG;
    if (slot < 0 || slot >= u->B || !phi_1 || !node_cond || !guess || !coarse_factor_ok(f) ||
        (long long)u->H * f > NX || (long long)u->W * f > NY || !(s_d != 0.f))
        return ufail(u, PIC_ERR_ARG, "pic_unet_coarse_guess: bad slot, pointer, factor, scale or grid");
    launch_cguess(u->out + (long long)slot * u->H * u->W, phi_1, phi_2, node_cond, NX, NY, periodic_x ? 1 : 0,
                  periodic_y ? 1 : 0, f, u->H, u->W, s_d, use_output ? 1 : 0, guess, u->stream);
    UCHK(u, hipGetLastError());
    return PIC_OK;
}

pic_status pic_solve_learned_coarse(pic_ctx *ctx, pic_unet *u, int32_t f, float s_r, float s_v, float s_d,
                                    double *guess, pic_solve_info *info)
{
    if (!ctx || !u) return PIC_ERR_ARG;
    if (u->B < 1) return PIC_ERR_ARG;
    PicCtxView v;
    pic_status st = pic_ctx_view(ctx, 0, &v);
    if (st != PIC_OK) return st;
    if (!guess || !coarse_factor_ok(f) || (long long)u->H * f > v.NX || (long long)u->W * f > v.NY)
        return ufail(u, PIC_ERR_ARG, "pic_solve_learned_coarse: factor, grid or guess");
    // the right-hand side and the potentials were written on the context's stream
    if ((st = after_stream(u, v.stream)) != PIC_OK) return st;
    launch_csample(v.b, v.phi, v.phi_prev, nullptr, v.node_cond, v.NX, v.NY, v.px, v.py, f, u->H, u->W, s_r, s_v,
                   s_d, u->x, nullptr, nullptr, nullptr, u->stream);
    if ((st = pic_unet_forward(u)) != PIC_OK) return st;
    launch_cguess(u->out, v.phi, v.phi_prev, v.node_cond, v.NX, v.NY, v.px, v.py, f, u->H, u->W, s_d, 1, guess,
                  u->stream);
    UCHK(u, hipGetLastError());
    UCHK(u, hipStreamSynchronize(u->stream));
    return pic_solve(ctx, 4, guess, info);
}

pic_status pic_unet_set_timing(pic_unet *u, int32_t on)
{
    if (!u) return PIC_ERR_ARG;
    if (on && !u->e0) {
        UCHK(u, hipEventCreate(&u->e0));
        UCHK(u, hipEventCreate(&u->e1));
    }
    u->timing = on != 0;
    return PIC_OK;
}

pic_status pic_unet_forward_timing(pic_unet *u, double *avg_ms, int32_t *passes)
{
    if (!u) return PIC_ERR_ARG;
    if (avg_ms) *avg_ms = u->timed_n ? u->timed_ms / u->timed_n : 0.0;
    if (passes) *passes = u->timed_n;
    u->timed_ms = 0.0;
    u->timed_n = 0;
    return PIC_OK;
}

void pic_unet_destroy(pic_unet *u)
{
    if (!u) return;
    if (u->e0) (void)hipEventDestroy(u->e0);
    if (u->e1) (void)hipEventDestroy(u->e1);
    delete u;
}

const char *pic_unet_last_error(const pic_unet *u) { return u ? u->err.c_str() : "null network"; }

} // extern "C"
