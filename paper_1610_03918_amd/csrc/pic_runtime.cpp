// Host runtime behind the C ABI of include/pic.h: validation, geometry
// (Dirichlet node map from the conductor cells), multigrid hierarchy,
// workspace carve-up, the solver's convergence loop and the step driver.
// Every device operation is a kernel from pic_kernels.hip on the caller's
// stream; the library allocates no device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "pic_internal.h"

using namespace pic;

namespace {

constexpr int kCoarseMaxNodes = 4096;   // largest level solved inside one work-group
constexpr int kCoarseMaxLds = 64 * 1024;
constexpr int kMaxTiming = 512;

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

struct Layout {
    int nx, ny, NX, NY, px, py;
    int nlev = 0;                           // multigrid levels (1 = none)
    int NXl[kMaxLev], NYl[kMaxLev];
    int lg = 0;                             // first level handled by the coarse kernel
    bool mg = false;
    int TX, TY, lx, ly, tiles_x, tiles_y, ntiles, H, chunk;
    int unroll, merge;                      // push kernel variant
    long long max_blocks[2];
    int grid_blocks;                        // blocks of the largest grid kernel
};

int ilog2(int v)
{
    int l = 0;
    while ((1 << l) < v) l++;
    return l;
}

bool coarsenable(int n, int periodic)
{
    return periodic ? (n % 2 == 0 && n >= 4) : (n % 2 == 1 && n >= 5);
}

int coarser(int n, int periodic) { return periodic ? n / 2 : (n + 1) / 2; }

std::string validate(const pic_config *c, const int64_t *cap)
{
    if (!c) return "null config";
    if (c->nx < 2 || c->ny < 2 || c->nx > 32767 || c->ny > 65535)
        return "grid size out of range (2..32767 x 2..65535 cells)";
    if (!(c->dt > 0)) return "dt must be positive";
    if (!c->cell_cond) return "cell_cond is required";
    for (int e = 0; e < 4; e++) {
        bool bounded = (e < 2) ? !c->periodic_x : !c->periodic_y;
        if (bounded && (c->edge_cond[e] <= 0 || c->edge_cond[e] >= PIC_MAX_COND))
            return "a bounded edge needs a conductor id in 1..7";
    }
    if (!(c->weight > 0)) return "weight must be positive";
    if (c->charge_mode < 0 || c->charge_mode > 2) return "charge_mode must be 0, 1 or 2";
    int NX = c->periodic_x ? c->nx : c->nx + 1;
    if (c->charge_mode && (c->charge_row < 0 || c->charge_row >= NX)) return "charge_row outside the grid";
    if (!(c->rtol > 0)) return "rtol must be positive";
    if (c->max_iter <= 0) return "max_iter must be positive";
    int tx = c->tile_x ? c->tile_x : 16, ty = c->tile_y ? c->tile_y : 16;
    if ((tx & (tx - 1)) || (ty & (ty - 1)) || tx > 256 || ty > 256) return "tile sizes must be powers of two <= 256";
    int H = c->halo ? c->halo : 4;
    if (H < 0 || H > 64) return "halo out of range";
    int chunk = c->chunk ? c->chunk : 8192;
    if (chunk < 256 || chunk > 8192) return "chunk must be in 256..8192";
    if (c->push_unroll != 0 && c->push_unroll != 1 && c->push_unroll != 2 && c->push_unroll != 4)
        return "push_unroll must be 0 (default), 1, 2 or 4";
    if (c->push_merge != 0 && c->push_merge != 2 && c->push_merge != 4)
        return "push_merge must be 0, 2 or 4";
    size_t lds = (size_t)(tx + 2 * H) * (ty + 2 * H) * 16 + 64;
    if (lds > 64 * 1024) return "tile + halo window exceeds 64 KiB of LDS";
    if (cap && (cap[0] < 0 || cap[1] < 0 || cap[0] > 0x7fffffffLL || cap[1] > 0x7fffffffLL))
        return "capacity out of range";
    if (c->hitlog_capacity < 0) return "hitlog_capacity must be >= 0";
    if (c->warm_start < 0 || c->warm_start > 1) return "warm_start must be 0 or 1";
    return "";
}

// Dirichlet map of the nodes: a node on a bounded edge takes the edge's
// conductor; a node touching a solid cell takes that cell's conductor.
// Returns false when two different conductors meet at one node.
bool node_map(const pic_config *c, std::vector<uint8_t> &nc)
{
    const int nx = c->nx, ny = c->ny, px = c->periodic_x, py = c->periodic_y;
    const int NX = px ? nx : nx + 1, NY = py ? ny : ny + 1;
    nc.assign((size_t)NX * NY, 0);
    bool ok = true;
    for (int i = 0; i < NX; i++)
        for (int j = 0; j < NY; j++) {
            int id = 0;
            auto put = [&](int v) {
                if (v <= 0) return;
                if (id && id != v) ok = false;
                if (!id) id = v;
            };
            if (!px && i == 0) put(c->edge_cond[0]);
            if (!px && i == nx) put(c->edge_cond[1]);
            if (!py && j == 0) put(c->edge_cond[2]);
            if (!py && j == ny) put(c->edge_cond[3]);
            for (int di = -1; di <= 0; di++)
                for (int dj = -1; dj <= 0; dj++) {
                    int a = i + di, b = j + dj;
                    if (px) a = (a + nx) % nx; else if (a < 0 || a >= nx) continue;
                    if (py) b = (b + ny) % ny; else if (b < 0 || b >= ny) continue;
                    put(c->cell_cond[(size_t)a * ny + b]);
                }
            nc[(size_t)i * NY + j] = (uint8_t)id;
        }
    return ok;
}

Layout make_layout(const pic_config *c, const int64_t *cap)
{
    Layout L;
    L.nx = c->nx;
    L.ny = c->ny;
    L.px = c->periodic_x ? 1 : 0;
    L.py = c->periodic_y ? 1 : 0;
    L.NX = L.px ? L.nx : L.nx + 1;
    L.NY = L.py ? L.ny : L.ny + 1;
    L.NXl[0] = L.NX;
    L.NYl[0] = L.NY;
    L.nlev = 1;
    while (L.nlev < kMaxLev && coarsenable(L.NXl[L.nlev - 1], L.px) &&
           coarsenable(L.NYl[L.nlev - 1], L.py)) {
        L.NXl[L.nlev] = coarser(L.NXl[L.nlev - 1], L.px);
        L.NYl[L.nlev] = coarser(L.NYl[L.nlev - 1], L.py);
        L.nlev++;
    }
    // coarse kernel takes every level from lg on; lg >= 1 and level lg must fit
    L.lg = 1;
    while (L.lg < L.nlev && L.NXl[L.lg] * L.NYl[L.lg] > kCoarseMaxNodes) L.lg++;
    L.mg = (c->solver == 0) && L.nlev >= 2 && L.lg < L.nlev;
    if (L.mg) {
        size_t lds = 0;
        for (int l = L.lg; l < L.nlev; l++) {
            size_t n = (size_t)L.NXl[l] * L.NYl[l];
            lds += ((n * 4 + 15) & ~size_t(15)) * 2 + ((n + 15) & ~size_t(15));
        }
        if (lds > kCoarseMaxLds) L.mg = false;
    }
    L.TX = c->tile_x ? c->tile_x : 16;
    L.TY = c->tile_y ? c->tile_y : 16;
    L.lx = ilog2(L.TX);
    L.ly = ilog2(L.TY);
    L.tiles_x = (L.nx + L.TX - 1) / L.TX;
    L.tiles_y = (L.ny + L.TY - 1) / L.TY;
    L.ntiles = L.tiles_x * L.tiles_y;
    L.H = c->halo ? c->halo : 4;
    L.chunk = c->chunk ? c->chunk : 8192;
    L.unroll = c->push_unroll ? c->push_unroll : 2;
    L.merge = c->push_merge;
    for (int s = 0; s < 2; s++) L.max_blocks[s] = L.ntiles + (cap[s] + L.chunk - 1) / L.chunk;
    int maxrows = std::max(L.NX, L.nx), maxcols = std::max(L.NY, L.ny);
    L.grid_blocks = ((maxcols + kGridBX - 1) / kGridBX) * ((maxrows + kGridBY - 1) / kGridBY);
    return L;
}

} // namespace

struct pic_ctx {
    pic_config cfg;
    std::vector<uint8_t> cell_cond;
    std::vector<uint8_t> node_cond;
    Layout L;
    Geom g;
    hipStream_t stream = nullptr;
    pic_buffers buf;
    int cur[2] = {0, 0};
    long long slots_ub[2] = {0, 0};
    long long loaded[2] = {0, 0};
    // workspace
    uint8_t *d_cell_cond = nullptr, *d_node_cond = nullptr;
    uint8_t *d_fix[kMaxLev] = {};
    float *d_u[kMaxLev] = {}, *d_g[kMaxLev] = {};
    float *d_e = nullptr, *d_p[2] = {}, *d_q = nullptr;
    double *d_phi_prev = nullptr;          // solution of the previous step (extrapolated start)
    bool have_prev = false;
    float4 *d_E4 = nullptr;
    double *d_part = nullptr, *d_S = nullptr;
    int *d_F = nullptr;
    unsigned *d_count = nullptr;
    unsigned *d_counts[2] = {}, *d_offsets[2] = {}, *d_cursor[2] = {}, *d_boff[2] = {};
    int4 *d_table[2] = {};
    long long *d_info[2] = {};
    unsigned long long *d_tally = nullptr, *d_surf = nullptr, *d_misc = nullptr;
    int32_t *d_hits = nullptr;
    CoarseArgs coarse;
    // state
    long long step = 0;
    int inner_chunk = 12;
    pic_solve_info last{};
    std::string err;
    // solver graphs: one outer pass (inner start, K iterations, phi update,
    // float64 residual) captured per K and replayed on the caller's stream
    hipStream_t cap_stream = nullptr;
    std::map<int, hipGraphExec_t> outer_graphs;
    bool use_graphs = true;
    double eta2_host = 0.0;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev0, ev1;
    int nev = 0;
    long long timed_particles = 0;
};

namespace {

pic_status fail(pic_ctx *c, pic_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

#define HIPCHK(ctx, call)                                                            \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return fail(ctx, PIC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Red red_of(pic_ctx *c)
{
    Red r;
    r.part = c->d_part;
    r.stride = c->L.grid_blocks;
    r.count = c->d_count;
    r.S = c->d_S;
    r.F = c->d_F;
    return r;
}

size_t carve(pic_ctx *c, const Layout &L, const pic_config *cfg, char *base)
{
    Carve w;
    w.base = base;
    const size_t cells = (size_t)L.nx * L.ny, nodes = (size_t)L.NX * L.NY;
    uint8_t *cc = w.take<uint8_t>(cells);
    uint8_t *nc = w.take<uint8_t>(nodes);
    uint8_t *fix[kMaxLev];
    float *u[kMaxLev], *gg[kMaxLev];
    for (int l = 0; l < L.nlev; l++) fix[l] = w.take<uint8_t>((size_t)L.NXl[l] * L.NYl[l]);
    for (int l = 0; l < L.nlev; l++) {
        u[l] = w.take<float>((size_t)L.NXl[l] * L.NYl[l]);
        gg[l] = w.take<float>((size_t)L.NXl[l] * L.NYl[l]);
    }
    float *e = w.take<float>(nodes), *p0 = w.take<float>(nodes), *p1 = w.take<float>(nodes);
    float *q = w.take<float>(nodes);
    float4 *E4 = w.take<float4>(2 * cells);
    double *phi_prev = w.take<double>(nodes);
    double *part = w.take<double>((size_t)L.grid_blocks * 2);
    double *S = w.take<double>(S_NSCAL);
    int *F = w.take<int>(F_NFLAG);
    unsigned *cnt = w.take<unsigned>(16);
    unsigned *counts[2], *offs[2], *curs[2], *boff[2];
    int4 *table[2];
    long long *info[2];
    for (int s = 0; s < 2; s++) {
        counts[s] = w.take<unsigned>(L.ntiles);
        offs[s] = w.take<unsigned>(L.ntiles);
        curs[s] = w.take<unsigned>(L.ntiles);
        boff[s] = w.take<unsigned>(L.ntiles);
        table[s] = w.take<int4>((size_t)L.max_blocks[s]);
        info[s] = w.take<long long>(8);
    }
    unsigned long long *tally = w.take<unsigned long long>(2 * kNClass);
    unsigned long long *surf = w.take<unsigned long long>(L.ny + 1);
    unsigned long long *misc = w.take<unsigned long long>(16);
    int32_t *hits = w.take<int32_t>((size_t)6 * std::max<int64_t>(cfg->hitlog_capacity, 1));
    if (c) {
        c->d_cell_cond = cc;
        c->d_node_cond = nc;
        for (int l = 0; l < L.nlev; l++) {
            c->d_fix[l] = fix[l];
            c->d_u[l] = u[l];
            c->d_g[l] = gg[l];
        }
        c->d_e = e;
        c->d_p[0] = p0;
        c->d_p[1] = p1;
        c->d_q = q;
        c->d_E4 = E4;
        c->d_phi_prev = phi_prev;
        c->d_part = part;
        c->d_S = S;
        c->d_F = F;
        c->d_count = cnt;
        for (int s = 0; s < 2; s++) {
            c->d_counts[s] = counts[s];
            c->d_offsets[s] = offs[s];
            c->d_cursor[s] = curs[s];
            c->d_boff[s] = boff[s];
            c->d_table[s] = table[s];
            c->d_info[s] = info[s];
        }
        c->d_tally = tally;
        c->d_surf = surf;
        c->d_misc = misc;
        c->d_hits = hits;
    }
    return w.off + 256;
}

LevelDev level(pic_ctx *c, int l)
{
    LevelDev d;
    d.NX = c->L.NXl[l];
    d.NY = c->L.NYl[l];
    d.u = c->d_u[l];
    d.g = c->d_g[l];
    d.fix = c->d_fix[l];
    return d;
}

void vtab(pic_ctx *c, double t, VTab &V)
{
    for (int k = 0; k < 8; k++) V.v[k] = 0.0;
    for (int k = 1; k < PIC_MAX_COND; k++)
        if (c->cfg.v_amp[k] != 0.0) V.v[k] = c->cfg.v_amp[k] * std::sin(c->cfg.v_omega[k] * t);
}

void enqueue_assemble(pic_ctx *c)
{
    VTab V;
    vtab(c, c->step * c->cfg.dt, V);
    const double q = std::ldexp(c->cfg.weight, -32);
    launch_assemble(c->g, c->d_node_cond, c->d_fix[0],
                    reinterpret_cast<const long long *>(c->buf.rho[0]),
                    reinterpret_cast<const long long *>(c->buf.rho[1]), q, V, c->cfg.charge_mode,
                    c->cfg.charge_row, c->d_surf, c->cfg.static_density, c->cfg.static_j_lo,
                    c->cfg.static_j_hi, c->buf.b, c->buf.phi, red_of(c), c->stream);
    if (c->g.px && c->g.py) launch_project_mean(c->g, c->d_fix[0], c->buf.b, red_of(c), c->stream);
}

PushArgs push_args(pic_ctx *c, int s)
{
    PushArgs a;
    a.g = c->g;
    a.TX = c->L.TX;
    a.TY = c->L.TY;
    a.lx = c->L.lx;
    a.ly = c->L.ly;
    a.tiles_y = c->L.tiles_y;
    a.H = c->L.H;
    a.WX = c->L.TX + 2 * c->L.H;
    a.WY = c->L.TY + 2 * c->L.H;
    a.cell_cond = c->d_cell_cond;
    a.E4 = c->d_E4;
    const int k = c->cur[s];
    a.cell = c->buf.sp[s].cell[k];
    a.ox = c->buf.sp[s].ox[k];
    a.oy = c->buf.sp[s].oy[k];
    a.vx = c->buf.sp[s].vx[k];
    a.vy = c->buf.sp[s].vy[k];
    a.table = c->d_table[s];
    a.info = c->d_info[s];
    a.rho = reinterpret_cast<unsigned long long *>(c->buf.rho[s]);
    a.qdt = (float)(c->cfg.alpha[s] * c->cfg.dt);
    a.dtf = (float)c->cfg.dt;
    a.box_i_top = c->cfg.box_i_top;
    a.box_j_lo = c->cfg.box_j_lo;
    a.box_j_hi = c->cfg.box_j_hi;
    a.species = s;
    a.tally = c->d_tally + s * kNClass;
    a.surf = (c->cfg.charge_mode == 2 && s == 1) ? c->d_surf : nullptr;
    a.log.rec = c->cfg.hitlog_capacity > 0 ? c->d_hits : nullptr;
    a.log.count = c->d_misc + 1;
    a.log.capacity = std::max<int64_t>(c->cfg.hitlog_capacity, 1);
    a.log.species_mask = c->cfg.hitlog_species_mask;
    a.step = (int)c->step;
    a.fallbacks = c->d_misc + 0;
    return a;
}

void enqueue_bin(pic_ctx *c, int s)
{
    BinArgs a;
    a.nx = c->L.nx;
    a.ny = c->L.ny;
    a.bad = c->d_misc + 2;
    a.lx = c->L.lx;
    a.ly = c->L.ly;
    a.tiles_y = c->L.tiles_y;
    a.ntiles = c->L.ntiles;
    a.chunk = c->L.chunk;
    const int src = c->cur[s], dst = 1 - src;
    const pic_species_buffers &B = c->buf.sp[s];
    a.cell = B.cell[src];
    a.ox = B.ox[src];
    a.oy = B.oy[src];
    a.vx = B.vx[src];
    a.vy = B.vy[src];
    a.cell2 = B.cell[dst];
    a.ox2 = B.ox[dst];
    a.oy2 = B.oy[dst];
    a.vx2 = B.vx[dst];
    a.vy2 = B.vy[dst];
    a.slots = c->d_info[s] + 2 + src;
    a.counts = c->d_counts[s];
    a.offsets = c->d_offsets[s];
    a.cursor = c->d_cursor[s];
    a.boff = c->d_boff[s];
    a.table = c->d_table[s];
    a.info = c->d_info[s];
    a.dst = dst;
    launch_bin(a, c->slots_ub[s], c->stream);
    c->cur[s] = dst;
}

void enqueue_deposit(pic_ctx *c)
{
    for (int s = 0; s < 2; s++)
        launch_zero_u64(reinterpret_cast<unsigned long long *>(c->buf.rho[s]),
                        (long long)c->g.NX * c->g.NY, c->stream);
    for (int s = 0; s < 2; s++) {
        PushArgs a = push_args(c, s);
        launch_push(a, (int)c->L.max_blocks[s], false, c->L.unroll, c->L.merge, c->stream);
    }
    enqueue_assemble(c);
}

// One V-cycle after the level-0 red-from-zero sweep (already applied).
void enqueue_vcycle_rest(pic_ctx *c)
{
    const Layout &L = c->L;
    Red r = red_of(c);
    const int *done = c->d_F + F_DONE;
    for (int l = 0; l < L.lg; l++) {
        launch_smooth(c->g, level(c, l), 1, 0, r, c->stream);
        launch_restrict(c->g, level(c, l), level(c, l + 1), done, c->stream);
    }
    launch_coarse(c->coarse, done, c->stream);
    for (int l = L.lg - 1; l >= 0; l--) {
        launch_prolong_black(c->g, level(c, l), level(c, l + 1), done, c->stream);
        launch_smooth(c->g, level(c, l), 0, l == 0 ? 1 : 0, r, c->stream);
    }
}

pic_status read_scalars(pic_ctx *c, double *S, int *F)
{
    HIPCHK(c, hipMemcpyAsync(S, c->d_S, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(F, c->d_F, sizeof(int) * F_NFLAG, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

// Kernels of one outer pass: inner preconditioned CG from e = 0 with K
// iterations (later ones return at once after the stop test), phi += e and
// the float64 residual with its norm.
void enqueue_outer(pic_ctx *c, int K, double eta2, hipStream_t st)
{
    Red r = red_of(c);
    LevelDev L0 = level(c, 0);
    const int mg = c->L.mg ? 1 : 0;
    const hipStream_t keep = c->stream;
    c->stream = st;
    launch_init_red0(c->g, L0, c->d_e, eta2, mg, r, st);
    if (mg) enqueue_vcycle_rest(c);
    for (int k = 0; k < K; k++) {
        const float *pold = c->d_p[k & 1];
        float *pnew = c->d_p[(k + 1) & 1];
        launch_pupdate_Ap(c->g, L0, pold, pnew, c->d_q, k == 0 ? 1 : 0, r, st);
        launch_update_red0(c->g, L0, pnew, c->d_q, c->d_e, mg, r, st);
        if (mg) enqueue_vcycle_rest(c);
    }
    launch_phi_update(c->g, c->d_fix[0], c->d_e, c->buf.phi, st);
    launch_resid64(c->g, c->d_fix[0], c->buf.b, c->buf.phi, L0.g, r, st);
    c->stream = keep;
}

int round_chunk(int k)
{
    static const int steps[] = {2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128};
    for (int v : steps)
        if (k <= v) return v;
    return k;
}

// The stop ratio of the inner solve is passed through S_ETA2 by a tiny copy
// so one captured graph serves every ratio.
pic_status run_outer(pic_ctx *c, int K, double eta2)
{
    if (!c->use_graphs || K > 128) {
        enqueue_outer(c, K, eta2, c->stream);
        HIPCHK(c, hipGetLastError());
        return PIC_OK;
    }
    auto it = c->outer_graphs.find(K);
    if (it == c->outer_graphs.end()) {
        if (!c->cap_stream)
            HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
        enqueue_outer(c, K, -1.0, c->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e1 = hipStreamEndCapture(c->cap_stream, &g);
        if (e1 != hipSuccess || !g) {
            c->use_graphs = false;
            (void)hipGetLastError();
            enqueue_outer(c, K, eta2, c->stream);
            return PIC_OK;
        }
        hipGraphExec_t ex = nullptr;
        hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) {
            c->use_graphs = false;
            (void)hipGetLastError();
            enqueue_outer(c, K, eta2, c->stream);
            return PIC_OK;
        }
        it = c->outer_graphs.emplace(K, ex).first;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_S + S_ETA2, &c->eta2_host, sizeof(double), hipMemcpyHostToDevice,
                             c->stream));
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    return PIC_OK;
}

pic_status do_solve(pic_ctx *c, int kind, const double *guess, pic_solve_info *info)
{
    Red r = red_of(c);
    LevelDev L0 = level(c, 0);
    if (kind == 0 || kind == 2)
        launch_set_guess(c->g, c->d_fix[0], kind, guess, c->buf.phi, c->stream);
    if (kind == 3) {
        launch_extrapolate(c->g, c->d_fix[0], c->buf.phi, c->d_phi_prev, c->have_prev ? 1 : 0,
                           c->stream);
        c->have_prev = true;
    } else {
        c->have_prev = false;
    }
    if (c->g.px && c->g.py) launch_pin_shift(c->g, c->buf.phi, r, c->stream);
    launch_resid64(c->g, c->d_fix[0], c->buf.b, c->buf.phi, L0.g, r, c->stream);
    double S[S_NSCAL];
    int F[F_NFLAG];
    pic_status st = read_scalars(c, S, F);
    if (st != PIC_OK) return st;
    const double bb = S[S_BB] > 0 ? S[S_BB] : 1.0;
    double relres = std::sqrt(S[S_RR64] / bb);
    pic_solve_info si{};
    si.relres0 = relres;
    int total = 0, outer = 0;
    const int mg = c->L.mg ? 1 : 0;
    while (relres > c->cfg.rtol && total < c->cfg.max_iter && outer < 64 && std::isfinite(relres)) {
        double eta = 0.3 * c->cfg.rtol / relres;
        eta = std::min(0.5, std::max(eta, mg ? 2e-6 : 1e-5));
        c->eta2_host = eta * eta;
        int K = std::max(1, std::min(c->inner_chunk, c->cfg.max_iter - total));
        K = round_chunk(K);
        st = run_outer(c, K, c->eta2_host);
        if (st != PIC_OK) return st;
        st = read_scalars(c, S, F);
        if (st != PIC_OK) return st;
        total += F[F_ITER];
        outer++;
        relres = std::sqrt(S[S_RR64] / bb);
        if (F[F_DONE]) c->inner_chunk = std::max(2, F[F_ITER] + 1);
        else c->inner_chunk = std::min(2 * K, mg ? 64 : 4096);
    }
    if (c->g.px && c->g.py) launch_shift_mean(c->g, c->buf.phi, r, c->stream);
    si.iterations = total;
    si.outer = outer;
    si.relres = relres;
    si.converged = relres <= c->cfg.rtol ? 1 : 0;
    c->last = si;
    if (info) *info = si;
    if (!si.converged) {
        char msg[160];
        snprintf(msg, sizeof msg, "solver stopped at relative residual %.3e after %d iterations",
                 relres, total);
        return fail(c, PIC_ERR_NOT_CONVERGED, msg);
    }
    return PIC_OK;
}

pic_status do_push(pic_ctx *c)
{
    launch_field(c->g, c->d_node_cond, c->buf.phi, c->d_E4,
                 reinterpret_cast<unsigned long long *>(c->buf.rho[0]),
                 reinterpret_cast<unsigned long long *>(c->buf.rho[1]), c->stream);
    for (int s = 0; s < 2; s++) {
        PushArgs a = push_args(c, s);
        const bool tm = c->timing && c->nev < kMaxTiming;
        if (tm) HIPCHK(c, hipEventRecord(c->ev0[c->nev], c->stream));
        launch_push(a, (int)c->L.max_blocks[s], true, c->L.unroll, c->L.merge, c->stream);
        if (tm) {
            HIPCHK(c, hipEventRecord(c->ev1[c->nev], c->stream));
            c->nev++;
            c->timed_particles += c->slots_ub[s];
        }
    }
    HIPCHK(c, hipGetLastError());
    c->step++;
    enqueue_assemble(c);
    for (int s = 0; s < 2; s++) {
        const int K = c->cfg.sort_interval[s];
        if (K > 0 && c->step % K == 0) enqueue_bin(c, s);
    }
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

} // namespace

extern "C" {

const char *pic_version(void) { return "pic-gfx950 1.0"; }

const char *pic_last_error(const pic_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pic_status pic_workspace_size(const pic_config *cfg, const int64_t *capacity, size_t *bytes)
{
    std::string v = validate(cfg, capacity);
    if (!v.empty() || !bytes || !capacity) return PIC_ERR_ARG;
    Layout L = make_layout(cfg, capacity);
    *bytes = carve(nullptr, L, cfg, nullptr);
    return PIC_OK;
}

pic_status pic_init(const pic_config *cfg, const pic_buffers *buf, void *stream, pic_ctx **out)
{
    if (!out) return PIC_ERR_ARG;
    *out = nullptr;
    pic_ctx *c = new (std::nothrow) pic_ctx();
    if (!c) return PIC_ERR_ARG;
    *out = c;
    if (!buf) return fail(c, PIC_ERR_ARG, "null buffers");
    const int64_t cap[2] = {buf->sp[0].capacity, buf->sp[1].capacity};
    std::string v = validate(cfg, cap);
    if (!v.empty()) return fail(c, PIC_ERR_ARG, v);
    for (int s = 0; s < 2; s++) {
        if (buf->sp[s].count < 0 || buf->sp[s].count > buf->sp[s].capacity)
            return fail(c, PIC_ERR_CAPACITY, "particle count exceeds capacity");
        for (int k = 0; k < 2; k++)
            if (buf->sp[s].capacity > 0 &&
                (!buf->sp[s].cell[k] || !buf->sp[s].ox[k] || !buf->sp[s].oy[k] ||
                 !buf->sp[s].vx[k] || !buf->sp[s].vy[k]))
                return fail(c, PIC_ERR_ARG, "missing particle buffer");
        if (!buf->rho[s]) return fail(c, PIC_ERR_ARG, "missing rho buffer");
    }
    if (!buf->phi || !buf->b || !buf->workspace) return fail(c, PIC_ERR_ARG, "missing phi, b or workspace");
    if (reinterpret_cast<uintptr_t>(buf->workspace) & 255)
        return fail(c, PIC_ERR_ARG, "workspace must be 256-byte aligned");
    c->cfg = *cfg;
    c->cell_cond.assign(cfg->cell_cond, cfg->cell_cond + (size_t)cfg->nx * cfg->ny);
    c->cfg.cell_cond = c->cell_cond.data();
    for (auto v8 : c->cell_cond)
        if (v8 >= PIC_MAX_COND) return fail(c, PIC_ERR_ARG, "cell conductor id above 7");
    if (!node_map(&c->cfg, c->node_cond))
        return fail(c, PIC_ERR_ARG, "two different conductors meet at a node");
    c->L = make_layout(&c->cfg, cap);
    const Layout &L = c->L;
    size_t need = carve(nullptr, L, &c->cfg, nullptr);
    if (buf->workspace_bytes < need) return fail(c, PIC_ERR_ARG, "workspace too small");
    carve(c, L, &c->cfg, reinterpret_cast<char *>(buf->workspace));
    c->buf = *buf;
    c->stream = reinterpret_cast<hipStream_t>(stream);
    c->g.nx = L.nx;
    c->g.ny = L.ny;
    c->g.NX = L.NX;
    c->g.NY = L.NY;
    c->g.px = L.px;
    c->g.py = L.py;

    // masks of every level: level 0 = Dirichlet nodes (plus node 0 pinned on a
    // fully periodic grid); coarse node fixed iff its coincident fine node is
    std::vector<std::vector<uint8_t>> fix(L.nlev);
    fix[0].resize((size_t)L.NX * L.NY);
    for (size_t n = 0; n < fix[0].size(); n++) fix[0][n] = c->node_cond[n] ? 1 : 0;
    if (L.px && L.py) fix[0][0] = 1;
    for (int l = 1; l < L.nlev; l++) {
        const int NXc = L.NXl[l], NYc = L.NYl[l], NYf = L.NYl[l - 1];
        fix[l].resize((size_t)NXc * NYc);
        for (int I = 0; I < NXc; I++)
            for (int J = 0; J < NYc; J++)
                fix[l][(size_t)I * NYc + J] = fix[l - 1][(size_t)(2 * I) * NYf + 2 * J];
    }
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(c->d_cell_cond, c->cell_cond.data(), c->cell_cond.size(),
                             hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_node_cond, c->node_cond.data(), c->node_cond.size(),
                             hipMemcpyHostToDevice, s));
    for (int l = 0; l < L.nlev; l++)
        HIPCHK(c, hipMemcpyAsync(c->d_fix[l], fix[l].data(), fix[l].size(), hipMemcpyHostToDevice, s));
    // coarse-kernel description
    CoarseArgs &ca = c->coarse;
    memset(&ca, 0, sizeof ca);
    if (L.mg) {
        ca.nlev = L.nlev - L.lg;
        int off = 0;
        for (int k = 0; k < ca.nlev; k++) {
            const int l = L.lg + k;
            const int n = L.NXl[l] * L.NYl[l];
            ca.NX[k] = L.NXl[l];
            ca.NY[k] = L.NYl[l];
            ca.off_u[k] = off;
            off += (n * 4 + 15) & ~15;
            ca.off_g[k] = off;
            off += (n * 4 + 15) & ~15;
            ca.off_f[k] = off;
            off += (n + 15) & ~15;
            ca.fix[k] = c->d_fix[l];
        }
        ca.lds_bytes = off;
        ca.u_top = c->d_u[L.lg];
        ca.g_top = c->d_g[L.lg];
        ca.px = L.px;
        ca.py = L.py;
        const int last = ca.nlev - 1;
        ca.sweeps = std::min(64, std::max(2, std::max(ca.NX[last], ca.NY[last])));
    }
    // zero counters and scalars
    HIPCHK(c, hipMemsetAsync(c->d_S, 0, sizeof(double) * S_NSCAL, s));
    HIPCHK(c, hipMemsetAsync(c->d_F, 0, sizeof(int) * F_NFLAG, s));
    HIPCHK(c, hipMemsetAsync(c->d_count, 0, sizeof(unsigned) * 16, s));
    HIPCHK(c, hipMemsetAsync(c->d_tally, 0, sizeof(unsigned long long) * 2 * kNClass, s));
    HIPCHK(c, hipMemsetAsync(c->d_surf, 0, sizeof(unsigned long long) * (L.ny + 1), s));
    HIPCHK(c, hipMemsetAsync(c->d_misc, 0, sizeof(unsigned long long) * 16, s));
    HIPCHK(c, hipMemsetAsync(c->d_e, 0, sizeof(float) * (size_t)L.NX * L.NY, s));
    HIPCHK(c, hipMemsetAsync(c->d_p[0], 0, sizeof(float) * (size_t)L.NX * L.NY, s));
    HIPCHK(c, hipMemsetAsync(c->buf.phi, 0, sizeof(double) * (size_t)L.NX * L.NY, s));
    for (int sp = 0; sp < 2; sp++) {
        long long info[8] = {0, 0, buf->sp[sp].count, 0, 0, 0, 0, 0};
        HIPCHK(c, hipMemcpyAsync(c->d_info[sp], info, sizeof info, hipMemcpyHostToDevice, s));
        c->cur[sp] = 0;
        c->slots_ub[sp] = buf->sp[sp].count;
        c->loaded[sp] = buf->sp[sp].count;
        // the copy above reads host memory: finish it before info goes out of scope
        HIPCHK(c, hipStreamSynchronize(s));
        enqueue_bin(c, sp);
    }
    c->ev0.resize(kMaxTiming);
    c->ev1.resize(kMaxTiming);
    for (int k = 0; k < kMaxTiming; k++) {
        HIPCHK(c, hipEventCreate(&c->ev0[k]));
        HIPCHK(c, hipEventCreate(&c->ev1[k]));
    }
    c->step = 0;
    enqueue_deposit(c);
    HIPCHK(c, hipGetLastError());
    unsigned long long bad = 0;
    HIPCHK(c, hipMemcpyAsync(&bad, c->d_misc + 2, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (bad) return fail(c, PIC_ERR_ARG, "particles with cell codes outside the grid");
    return PIC_OK;
}

pic_status pic_deposit(pic_ctx *c)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    enqueue_deposit(c);
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status pic_solve(pic_ctx *c, int32_t guess_kind, const double *guess, pic_solve_info *info)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    if (guess_kind < 0 || guess_kind > 3 || (guess_kind == 2 && !guess))
        return fail(c, PIC_ERR_ARG, "guess_kind must be 0, 1, 2 (with a guess array) or 3");
    return do_solve(c, guess_kind, guess, info);
}

pic_status pic_rewind(pic_ctx *c)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    launch_field(c->g, c->d_node_cond, c->buf.phi, c->d_E4, nullptr, nullptr, c->stream);
    for (int s = 0; s < 2; s++) {
        const int k = c->cur[s];
        const pic_species_buffers &B = c->buf.sp[s];
        launch_rewind(c->g, c->d_E4, B.cell[k], B.ox[k], B.oy[k], B.vx[k], B.vy[k], c->slots_ub[s],
                      c->d_info[s] + 2 + k, (float)(0.5 * c->cfg.alpha[s] * c->cfg.dt), c->stream);
    }
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status pic_push(pic_ctx *c)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    return do_push(c);
}

pic_status pic_step(pic_ctx *c, int32_t nsteps)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    if (nsteps < 0) return fail(c, PIC_ERR_ARG, "nsteps < 0");
    for (int k = 0; k < nsteps; k++) {
        pic_status st = do_solve(c, c->cfg.warm_start == 1 ? 3 : 1, nullptr, nullptr);
        if (st != PIC_OK) return st;
        st = do_push(c);
        if (st != PIC_OK) return st;
    }
    return PIC_OK;
}

pic_status pic_sort(pic_ctx *c, int32_t species)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    if (species < 0 || species > 1) return fail(c, PIC_ERR_ARG, "species must be 0 or 1");
    enqueue_bin(c, species);
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status pic_diagnostics(pic_ctx *c, pic_diag *out)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    if (!out) return fail(c, PIC_ERR_ARG, "null output");
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemsetAsync(c->d_misc + 4, 0, 2 * sizeof(unsigned long long), s));
    for (int sp = 0; sp < 2; sp++)
        launch_rho_sum(reinterpret_cast<const unsigned long long *>(c->buf.rho[sp]),
                       (long long)c->g.NX * c->g.NY, c->d_misc + 4 + sp, s);
    unsigned long long tally[2 * kNClass], misc[16];
    std::vector<unsigned long long> surf(c->L.ny + 1);
    HIPCHK(c, hipMemcpyAsync(tally, c->d_tally, sizeof tally, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(misc, c->d_misc, sizeof misc, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(surf.data(), c->d_surf, surf.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    memset(out, 0, sizeof *out);
    out->step = c->step;
    out->t = c->step * c->cfg.dt;
    for (int sp = 0; sp < 2; sp++) {
        long long lost = 0;
        for (int k = 0; k < kNClass; k++) {
            out->tally[sp][k] = (int64_t)tally[sp * kNClass + k];
            lost += (long long)tally[sp * kNClass + k];
        }
        out->loaded[sp] = c->loaded[sp];
        out->alive[sp] = c->loaded[sp] - lost;
        out->charge[sp] = (int64_t)misc[4 + sp];
    }
    long long sh = 0;
    for (auto v8 : surf) sh += (long long)v8;
    out->surf_hits = sh;
    out->hits_logged = (int64_t)misc[1];
    out->deposit_fallbacks = (int64_t)misc[0];
    out->last_solve = c->last;
    return PIC_OK;
}

pic_status pic_particles(pic_ctx *c, int32_t species, int32_t *set, int64_t *slots)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    if (species < 0 || species > 1) return fail(c, PIC_ERR_ARG, "species must be 0 or 1");
    long long info[8];
    HIPCHK(c, hipMemcpyAsync(info, c->d_info[species], sizeof info, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (set) *set = c->cur[species];
    if (slots) *slots = info[2 + c->cur[species]];
    return PIC_OK;
}

pic_status pic_read_hits(pic_ctx *c, pic_hit *out, int64_t max, int64_t *n)
{
    if (!c || !c->d_E4) return fail(c, PIC_ERR_STATE, "not initialised");
    if (!out || !n || max < 0) return fail(c, PIC_ERR_ARG, "bad output");
    *n = 0;
    if (c->cfg.hitlog_capacity <= 0) return PIC_OK;
    unsigned long long total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, c->d_misc + 1, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const long long cap = c->cfg.hitlog_capacity;
    long long have = (long long)std::min<unsigned long long>(total, (unsigned long long)cap);
    long long take = std::min<long long>(have, max);
    std::vector<int32_t> all((size_t)cap * 6);
    HIPCHK(c, hipMemcpyAsync(all.data(), c->d_hits, all.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // oldest of the kept records first
    long long first = (long long)total - take;
    for (long long k = 0; k < take; k++) {
        long long slot = (first + k) % cap;
        memcpy(&out[k], &all[(size_t)slot * 6], sizeof(pic_hit));
    }
    *n = take;
    return PIC_OK;
}

pic_status pic_set_timing(pic_ctx *c, int32_t on)
{
    if (!c) return PIC_ERR_STATE;
    c->timing = on != 0;
    c->nev = 0;
    c->timed_particles = 0;
    return PIC_OK;
}

pic_status pic_push_timing(pic_ctx *c, double *avg_ms, double *avg_particles, int32_t *launches)
{
    if (!c) return PIC_ERR_STATE;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (int k = 0; k < c->nev; k++) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev0[k], c->ev1[k]));
        tot += ms;
    }
    if (avg_ms) *avg_ms = c->nev ? tot / c->nev : 0.0;
    if (avg_particles) *avg_particles = c->nev ? (double)c->timed_particles / c->nev : 0.0;
    if (launches) *launches = c->nev;
    c->nev = 0;
    c->timed_particles = 0;
    return PIC_OK;
}

void pic_destroy(pic_ctx *c)
{
    if (!c) return;
    if (c->d_E4) (void)hipStreamSynchronize(c->stream);
    for (auto &kv : c->outer_graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto e : c->ev0) if (e) (void)hipEventDestroy(e);
    for (auto e : c->ev1) if (e) (void)hipEventDestroy(e);
    delete c;
}

} // extern "C"
