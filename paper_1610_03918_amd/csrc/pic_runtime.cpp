// Host runtime behind the C ABI of include/pic.h: validation, geometry
// (Dirichlet node map from the conductor cells), multigrid hierarchy,
// workspace carve-up, launch tables of a batch of instances, the solver's
// convergence loop, the step driver and graph-captured multi-step launches.
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
#include "ctx_view.h"
#include "pic_internal.h"

using namespace pic;

namespace {

constexpr int kCoarseMaxNodes = 12288;  // largest level solved inside one work-group
constexpr int kCoarseMaxLds = 159 * 1024;   // dynamic LDS of the coarse kernel (160 KiB per work-group)
constexpr int kDenseTruncNodes = 256;       // coarsest level at most this size (see make_layout)
constexpr int kMaxTiming = 512;

struct Layout {
    int nx, ny, NX, NY, px, py;
    int nlev = 0;                           // multigrid levels (1 = none)
    int NXl[kMaxLev], NYl[kMaxLev];
    int lg = 0;                             // first level handled by the coarse kernel
    bool mg = false;
    int dense_n = 0;                        // nodes of a coarsest level solved with its inverse (0: sweeps)
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

// Status of a validation message: PIC_ERR_OVERFLOW for the fixed-point
// charge bound, PIC_ERR_ARG otherwise.
pic_status validate_status(const std::string &v)
{
    return v.rfind("charge overflow", 0) == 0 ? PIC_ERR_OVERFLOW : PIC_ERR_ARG;
}

// Secondary electron emission at the trench surfaces is on.
bool see_on(const pic_config *c) { return c->see_yield[0] > 0.0 || c->see_yield[1] > 0.0; }

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
    if (c->solver < 0 || c->solver > 3) return "solver must be 0 (MG-CG), 1 (CG), 2 (Jacobi) or 3 (Gauss-Seidel)";
    if (c->solver == 3 && ((c->periodic_x && (c->nx & 1)) || (c->periodic_y && (c->ny & 1))))
        return "red-black Gauss-Seidel needs an even node count on a periodic axis";
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
    if (push_lds_bytes(tx, ty, H) > 64 * 1024) return "tile + halo window exceeds 64 KiB of LDS";
    if (cap && (cap[0] < 0 || cap[1] < 0)) return "capacity out of range";
    if (cap && (cap[0] > 0x7fffffffLL || cap[1] > 0x7fffffffLL))
        return "charge overflow: a capacity above 2^31 - 1 particles could exceed the int64 charge of a node "
               "(2^32 units per particle)";
    if (c->hitlog_capacity < 0) return "hitlog_capacity must be >= 0";
    if (c->warm_start < 0 || c->warm_start > 1) return "warm_start must be 0 or 1";
    if (c->recycle_rows < 0 || c->recycle_rows > c->nx) return "recycle_rows must be in 0 .. nx";
    if (c->recycle_rows > 0 && !(c->recycle_vth >= 0)) return "recycle_vth must be >= 0";
    if (c->cell_cond)
        for (size_t q = 0; q < (size_t)c->recycle_rows * c->ny; q++)
            if (c->cell_cond[q]) return "the recycling rows must hold no solid cell";
    for (int s = 0; s < 2; s++)
        if (!(c->see_yield[s] >= 0.0 && c->see_yield[s] <= 1.0)) return "see_yield must be in 0 .. 1";
    if (see_on(c)) {
        if (!(c->see_vth > 0.0)) return "see_vth must be positive with a secondary-emission yield";
        if (c->hitlog_capacity < 65536)
            return "secondary emission reads the hit ring: hitlog_capacity must be at least 65536";
        for (int s = 0; s < 2; s++)
            if (c->see_yield[s] > 0.0 && !((c->hitlog_species_mask >> s) & 1))
                return "secondary emission: hitlog_species_mask must log every species with a yield";
    }
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
    // coarse kernel takes every level from lg on: the first level from 1 on
    // within kCoarseMaxNodes whose levels fit in the kernel's LDS together
    auto lds_from = [&](int lg) {
        size_t lds = 0;
        for (int l = lg; l < L.nlev; l++) {
            size_t n = (size_t)L.NXl[l] * L.NYl[l];
            lds += ((n * 4 + 15) & ~size_t(15)) * 2 + ((n + 15) & ~size_t(15));
        }
        if (lg < L.nlev) lds += ((size_t)L.NXl[lg] * L.NYl[lg] * 4 + 15) & ~size_t(15);   // scratch
        return lds;
    };
    L.lg = 1;
    while (L.lg < L.nlev && (L.NXl[L.lg] * L.NYl[L.lg] > kCoarseMaxNodes || lds_from(L.lg) > kCoarseMaxLds)) L.lg++;
    L.mg = (c->solver == 0) && L.nlev >= 2 && L.lg < L.nlev;
    // the hierarchy stops at the first level below the coarse kernel's first
    // that has at most kDenseTruncNodes nodes: solved exactly (below), it costs
    // one memory latency, where each further level costs a chain of
    // single-wavefront passes
    if (L.mg)
        for (int l = L.lg + 1; l < L.nlev; l++)
            if (L.NXl[l] * L.NYl[l] <= kDenseTruncNodes) {
                L.nlev = l + 1;
                break;
            }
    // the coarsest level is solved exactly with its inverse rather than swept
    // (a periodic axis with an odd factor stops the coarsening early, and a
    // large coarsest level needs many sweeps) when it is small enough and its
    // column partial sums fit in the coarse kernel's LDS
    if (L.mg) {
        const int last = L.nlev - 1, n = L.NXl[last] * L.NYl[last];
        const size_t part = ((size_t)kCoarseWaves * n * 4 + 15) & ~size_t(15);
        if (n <= kDenseMaxNodes && lds_from(L.lg) + part <= (size_t)kCoarseMaxLds) L.dense_n = n;
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
    L.unroll = c->push_unroll ? c->push_unroll : 4;
    L.merge = c->push_merge;
    for (int s = 0; s < 2; s++) L.max_blocks[s] = L.ntiles + (cap[s] + L.chunk - 1) / L.chunk;
    // appended electrons (secondary emission) get blocks of their own after
    // the binned ones: at most two more than a full binning would need
    if (see_on(c)) L.max_blocks[0] += 2;
    int maxrows = std::max(L.NX, L.nx), maxcols = std::max(L.NY, L.ny);
    L.grid_blocks = ((maxcols + kGridBX - 1) / kGridBX) * ((maxrows + kGridBY - 1) / kGridBY);
    return L;
}

} // namespace

// ---------------------------------------------------------------------------
// host-side state
// ---------------------------------------------------------------------------

namespace {

struct InstHost {
    pic_config cfg{};
    std::vector<uint8_t> cell_cond, node_cond;
    Layout L{};
    Geom g{};
    pic_buffers buf{};
    long long loaded[2] = {0, 0};
    long long slots_ub[2] = {0, 0};
    uint8_t *d_cell_cond = nullptr, *d_node_cond = nullptr;
    uint8_t *d_fix[kMaxLev] = {};
    float *d_u[kMaxLev] = {}, *d_g[kMaxLev] = {}, *d_uo[kMaxLev] = {};
    float *d_e = nullptr, *d_p[2] = {}, *d_q = nullptr;
    float *d_cg_r1 = nullptr, *d_cg_s[2] = {}, *d_cg_w = nullptr;
    float4 *d_E4 = nullptr;
    double *d_phi_prev = nullptr, *d_phi2 = nullptr;
    unsigned *d_counts[2] = {}, *d_offsets[2] = {}, *d_cursor[2] = {}, *d_boff[2] = {};
    int4 *d_table[2] = {};
    long long *d_info[2] = {};
    unsigned long long *d_tally = nullptr, *d_surf = nullptr, *d_misc = nullptr, *d_iad = nullptr;
    double *d_diag = nullptr;
    int32_t *d_hits = nullptr;
    std::vector<std::vector<uint8_t>> fixh;  // level masks (host copies kept until uploaded)
    std::vector<float> ainvh;               // coarsest-level inverse (host copy kept until uploaded)
    float *d_ainv = nullptr;
    bool dense = false;                     // the coarsest level is solved with d_ainv
    Inst dev{};
    pic_solve_info last{};
};

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

constexpr int kVWindow = 512;   // steps of conductor potentials held on the device
constexpr int kContinueChunk = 64; // inner iterations per graph between stop tests (plain CG)

} // namespace

struct pic_ctx {
    int n = 0;
    bool device_error = false;      // a device error bit was seen: every later call fails
    std::vector<InstHost> in;
    hipStream_t stream = nullptr;
    // shared device objects
    Inst *d_inst = nullptr;
    PushArgs *d_push = nullptr;
    BinArgs *d_bin = nullptr;
    double *d_part = nullptr;
    int part_stride = 0;
    double *d_S = nullptr;          // n x S_NSCAL
    int *d_F = nullptr;             // n x F_NFLAG
    char *h_flags = nullptr;       // pinned host copy of the span d_S .. end of d_F
    size_t flags_bytes = 0;
    double *d_V = nullptr;          // kVWindow x n x 8
    long long *d_ctl = nullptr;     // [0] step, [1] first step of the V window
    long long step = 0, vbase = 0;
    std::vector<double> vhost;
    // launch tables
    Tab t_l0{}, t_field{}, t_per{}, t_coarse{}, t_push{}, t_rewind{};
    Tab t_recycle{};                // ion units with recycling: one thread per slot
    Tab t_see{}, t_see1{};          // instances with secondary emission: kEmitBlocks blocks / one
    SeeArgs *d_see = nullptr;
    Tab t_plain{};                 // level-0 grid of the instances solved by plain CG
    Tab t_fine[kMaxLev] = {};      // 32 x 32 tiles of the fine multigrid levels handled one at a time
    Tab t_pair[kMaxLev] = {};      // 32 x 32 tiles of level l + 1 for levels l, l + 1 in one launch
    int maxlg = 0, coarse_lds = 0, any_mg = 0;
    int pair_levels = 1;           // fine levels 1, 2 (3, 4, ...) two per launch
    size_t push_lds = 0;
    int unroll = 2, merge = 0;
    // solver control
    bool have_prev = false;
    int pass_chunk[2] = {12, 12};   // inner iterations per pass (first pass, later passes)
    // re-binning inside pic_step: queued on a stream of its own behind the
    // push, so that it runs beside the next step's solve (which leaves most
    // CUs idle); the next push, and every entry point, waits for it
    hipStream_t bin_stream = nullptr;
    hipEvent_t ev_bin_go = nullptr, ev_bin_done = nullptr;
    bool bin_pending = false;
    // graphs
    hipStream_t cap_stream = nullptr;
    std::map<int, hipGraphExec_t> outer_graphs;   // CG passes by K; sweep chunks by kSweepKey + count
    int sweep_solver = 0;          // 2 Jacobi, 3 Gauss-Seidel (every instance), 0 CG
    std::map<int, hipGraphExec_t> chunk_graphs;
    std::map<long long, hipGraphExec_t> step_graphs;
    bool use_graphs = true;
    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev0, ev1;
    int nev = 0;
    long long timed_particles = 0;
    std::string err;
};

namespace {

pic_status fail(pic_ctx *c, pic_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, PIC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

Part part_of(pic_ctx *c) { return Part{c->d_part, c->part_stride}; }

int grid_blocks(int NX, int NY) { return ((NY + kGridBX - 1) / kGridBX) * ((NX + kGridBY - 1) / kGridBY); }

void tab_add_grid(Tab &t, int id, int NX, int NY)
{
    const int k = t.n++;
    t.id[k] = id;
    t.bx[k] = (NY + kGridBX - 1) / kGridBX;
    t.boff[k + 1] = t.boff[k] + t.bx[k] * ((NX + kGridBY - 1) / kGridBY);
}

void tab_add(Tab &t, int id, int blocks)
{
    const int k = t.n++;
    t.id[k] = id;
    t.bx[k] = 1;
    t.boff[k + 1] = t.boff[k] + blocks;
}

// Inverse of the coarsest level's operator, 4 u_k minus the free neighbours'
// u (periodic wrap as the kernels take it) on free nodes, u = 0 on fixed
// ones: float64 Cholesky factor, then one column of the inverse per free
// node.  Stored as the packed lower triangle (tri_off) in float32, zero in
// the rows and columns of fixed nodes, its diagonal halved: the kernel's
// row sums and column sums each take half of it.
// False when the operator is singular or nearly so (no fixed node).
bool coarse_inverse(const std::vector<uint8_t> &fix, int NX, int NY, std::vector<float> &out)
{
    const int n = NX * NY;
    std::vector<int> idx(n, -1), node;
    for (int k = 0; k < n; k++)
        if (!fix[k]) {
            idx[k] = (int)node.size();
            node.push_back(k);
        }
    const int m = (int)node.size();
    if (m == 0) return false;
    std::vector<double> A((size_t)m * m, 0.0);
    for (int a = 0; a < m; a++) {
        const int i = node[a] / NY, j = node[a] % NY;
        A[(size_t)a * m + a] = 4.0;
        const int nb[4] = {((i + NX - 1) % NX) * NY + j, ((i + 1) % NX) * NY + j, i * NY + (j + NY - 1) % NY,
                           i * NY + (j + 1) % NY};
        for (int q = 0; q < 4; q++)
            if (idx[nb[q]] >= 0) A[(size_t)a * m + idx[nb[q]]] -= 1.0;
    }
    for (int p = 0; p < m; p++) {                 // lower factor in place: A = L L^T
        double *rp = &A[(size_t)p * m];
        double d = rp[p];
        for (int q = 0; q < p; q++) d -= rp[q] * rp[q];
        if (!(d > 1e-8)) return false;              // singular to rounding (no fixed node)
        d = std::sqrt(d);
        rp[p] = d;
        for (int r = p + 1; r < m; r++) {
            double *rr = &A[(size_t)r * m];
            double v = rr[p];
            for (int q = 0; q < p; q++) v -= rr[q] * rp[q];
            rr[p] = v / d;
        }
    }
    std::vector<double> LT((size_t)m * m);        // L^T, for the backward substitutions
    for (int r = 0; r < m; r++)
        for (int q = 0; q <= r; q++) LT[(size_t)q * m + r] = A[(size_t)r * m + q];
    out.assign((size_t)tri_off(n), 0.0f);
    std::vector<double> x(m);
    for (int cidx = 0; cidx < m; cidx++) {
        std::fill(x.begin(), x.end(), 0.0);
        x[cidx] = 1.0;
        for (int r = cidx; r < m; r++) {           // L y = e_c (y is 0 above c)
            const double *rr = &A[(size_t)r * m];
            double v = x[r];
            for (int q = cidx; q < r; q++) v -= rr[q] * x[q];
            x[r] = v / rr[r];
        }
        for (int r = m - 1; r >= 0; r--) {         // L^T x = y
            const double *tr = &LT[(size_t)r * m];
            double v = x[r];
            for (int q = r + 1; q < m; q++) v -= tr[q] * x[q];
            x[r] = v / tr[r];
        }
        const int cn = node[cidx];
        for (int r = 0; r < m; r++) {
            const int rn = node[r];
            if (rn > cn) out[(size_t)tri_off(rn) + cn] = (float)x[r];
            else if (rn == cn) out[(size_t)tri_off(rn) + cn] = (float)(0.5 * x[r]);
        }
    }
    return true;
}

// Per-instance device memory inside the shared workspace.
void carve_inst(InstHost *h, Carve &w, const Layout &L, const pic_config *cfg, const int64_t *cap)
{
    const size_t cells = (size_t)L.nx * L.ny, nodes = (size_t)L.NX * L.NY;
    uint8_t *cc = w.take<uint8_t>(cells);
    uint8_t *nc = w.take<uint8_t>(nodes);
    uint8_t *fix[kMaxLev];
    float *u[kMaxLev], *gg[kMaxLev], *uo[kMaxLev] = {};
    for (int l = 0; l < L.nlev; l++) fix[l] = w.take<uint8_t>((size_t)L.NXl[l] * L.NYl[l]);
    for (int l = 0; l < L.nlev; l++) {
        u[l] = w.take<float>((size_t)L.NXl[l] * L.NYl[l]);
        gg[l] = w.take<float>((size_t)L.NXl[l] * L.NYl[l]);
        // fine multigrid levels keep the down half-cycle's result apart from its input
        if (L.mg && l < L.lg) uo[l] = w.take<float>((size_t)L.NXl[l] * L.NYl[l]);
    }
    float *e = w.take<float>(nodes), *p0 = w.take<float>(nodes), *p1 = w.take<float>(nodes);
    float *q = w.take<float>(nodes);
    // multigrid-preconditioned CG: second residual buffer, the s pair, w
    float *cg[4] = {};
    if (L.mg)
        for (int k = 0; k < 4; k++) cg[k] = w.take<float>(nodes);
    float4 *E4 = w.take<float4>(2 * cells);
    double *phi_prev = w.take<double>(nodes);
    double *phi2 = cfg->solver == 2 ? w.take<double>(nodes) : nullptr;
    float *ainv = L.dense_n ? w.take<float>((size_t)tri_off(L.dense_n)) : nullptr;
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
    unsigned long long *iad = w.take<unsigned long long>(kIadBins);
    double *diag = w.take<double>(kDiagBlocks + 4);
    int32_t *hits = w.take<int32_t>((size_t)6 * std::max<int64_t>(cfg->hitlog_capacity, 1));
    (void)cap;
    if (!h) return;
    h->d_cell_cond = cc;
    h->d_node_cond = nc;
    h->d_ainv = ainv;
    for (int l = 0; l < L.nlev; l++) {
        h->d_fix[l] = fix[l];
        h->d_u[l] = u[l];
        h->d_g[l] = gg[l];
        h->d_uo[l] = uo[l] ? uo[l] : u[l];
    }
    h->d_e = e;
    h->d_p[0] = p0;
    h->d_p[1] = p1;
    h->d_q = q;
    h->d_cg_r1 = cg[0];
    h->d_cg_s[0] = cg[1];
    h->d_cg_s[1] = cg[2];
    h->d_cg_w = cg[3];
    h->d_E4 = E4;
    h->d_phi_prev = phi_prev;
    h->d_phi2 = phi2;
    for (int s = 0; s < 2; s++) {
        h->d_counts[s] = counts[s];
        h->d_offsets[s] = offs[s];
        h->d_cursor[s] = curs[s];
        h->d_boff[s] = boff[s];
        h->d_table[s] = table[s];
        h->d_info[s] = info[s];
    }
    h->d_tally = tally;
    h->d_surf = surf;
    h->d_misc = misc;
    h->d_iad = iad;
    h->d_diag = diag;
    h->d_hits = hits;
}

// Whole workspace: shared part, then every instance.
size_t carve_all(pic_ctx *c, int n, const pic_config *cfgs, const int64_t *caps, char *base)
{
    Carve w;
    w.base = base;
    int stride = 0;
    for (int k = 0; k < n; k++) {
        Layout L = make_layout(&cfgs[k], caps + 2 * k);
        const int tiles0 = ((L.NX + kMgTileHost - 1) / kMgTileHost) * ((L.NY + kMgTileHost - 1) / kMgTileHost);
        stride += std::max(grid_blocks(std::max(L.NX, L.nx), std::max(L.NY, L.ny)), tiles0);
    }
    Inst *di = w.take<Inst>(n);
    PushArgs *dp = w.take<PushArgs>(2 * n);
    BinArgs *db = w.take<BinArgs>(2 * n);
    SeeArgs *dse = w.take<SeeArgs>(n);
    // partials of block reductions: two quantities, then the level-0 up
    // kernel's two (kept for the next level-0 down kernel)
    double *part = w.take<double>((size_t)4 * stride);
    double *S = w.take<double>((size_t)n * S_NSCAL);
    int *F = w.take<int>((size_t)n * F_NFLAG);
    double *V = w.take<double>((size_t)kVWindow * n * 8);
    long long *ctl = w.take<long long>(4);
    if (c) {
        c->d_inst = di;
        c->d_push = dp;
        c->d_bin = db;
        c->d_see = dse;
        c->d_part = part;
        c->part_stride = stride;
        c->d_S = S;
        c->d_F = F;
        c->d_V = V;
        c->d_ctl = ctl;
    }
    for (int k = 0; k < n; k++) {
        Layout L = make_layout(&cfgs[k], caps + 2 * k);
        carve_inst(c ? &c->in[k] : nullptr, w, L, &cfgs[k], caps + 2 * k);
    }
    return w.off + 256;
}

void fill_vwindow(pic_ctx *c, long long first)
{
    c->vbase = first;
    c->vhost.assign((size_t)kVWindow * c->n * 8, 0.0);
    for (long long s = 0; s < kVWindow; s++) {
        for (int k = 0; k < c->n; k++) {
            const pic_config &cf = c->in[k].cfg;
            const double t = (double)(first + s) * cf.dt;
            double *v = &c->vhost[((size_t)s * c->n + k) * 8];
            for (int q = 1; q < PIC_MAX_COND; q++)
                if (cf.v_amp[q] != 0.0) v[q] = cf.v_amp[q] * std::sin(cf.v_omega[q] * t);
        }
    }
}

// Uploads the potentials of steps [first, first + kVWindow) and the device
// step counter / window start.
pic_status upload_vwindow(pic_ctx *c, long long first)
{
    HIPCHK(c, hipStreamSynchronize(c->stream));
    fill_vwindow(c, first);
    long long ctl[2] = {c->step, c->vbase};
    HIPCHK(c, hipMemcpyAsync(c->d_V, c->vhost.data(), c->vhost.size() * sizeof(double),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_ctl, ctl, sizeof ctl, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PIC_OK;
}

// Keeps steps [from, from + ahead] inside the device window of potentials.
pic_status ensure_vwindow(pic_ctx *c, long long from, long long ahead)
{
    if (from >= c->vbase && from + ahead < c->vbase + kVWindow) return PIC_OK;
    return upload_vwindow(c, from);
}

void enqueue_assemble(pic_ctx *c, hipStream_t s)
{
    launch_assemble(c->d_inst, c->t_l0, c->d_V, c->d_ctl, c->n, kVWindow, part_of(c), s);
    launch_project_mean(c->d_inst, c->t_per, part_of(c), s);
}

// Tabs over (instance, species) pairs selected by mask bits (bit s: species s).
void bin_tabs(pic_ctx *c, int species_mask, Tab &tc, Tab &ts, Tab &tt)
{
    tc = Tab{};
    ts = Tab{};
    tt = Tab{};
    for (int k = 0; k < c->n; k++)
        for (int s = 0; s < 2; s++) {
            if (!((species_mask >> s) & 1)) continue;
            const InstHost &h = c->in[k];
            const int id = 2 * k + s;
            tab_add(tc, id, (int)((h.slots_ub[s] + bin_per_block() - 1) / bin_per_block()));
            tab_add(ts, id, 1);
            tab_add(tt, id, (h.L.ntiles + 255) / 256);
        }
}

void enqueue_bin(pic_ctx *c, int species_mask, hipStream_t s)
{
    Tab tc, ts, tt;
    bin_tabs(c, species_mask, tc, ts, tt);
    launch_bin(c->d_bin, tc, ts, tt, s);
}

void enqueue_deposit(pic_ctx *c, hipStream_t s)
{
    for (auto &h : c->in)
        for (int sp = 0; sp < 2; sp++)
            launch_zero_u64(reinterpret_cast<unsigned long long *>(h.buf.rho[sp]),
                            (long long)h.g.NX * h.g.NY, s);
    launch_push(c->d_push, c->t_push, false, c->unroll, c->merge, c->push_lds, s);
    enqueue_assemble(c, s);
}

// Levels 1 .. of a V-cycle: down half-cycles, the LDS levels, up
// half-cycles (level 0's halves carry the CG step and its dot products).
void enqueue_vcycle_mid(pic_ctx *c, bool fuse_update, hipStream_t s)
{
    Part pt = part_of(c);
    for (int l = 1; l < c->maxlg; l++) {
        launch_mg_pair(c->d_inst, c->t_pair[l], l, true, s);
        launch_mg_down(c->d_inst, c->t_fine[l], l, 0, 0, pt, s);
    }
    launch_coarse(c->d_inst, c->t_coarse, c->coarse_lds, c->t_fine[0], pt, fuse_update, s);
    for (int l = c->maxlg - 1; l >= 1; l--) {
        launch_mg_up(c->d_inst, c->t_fine[l], l, 0, pt, s);
        launch_mg_pair(c->d_inst, c->t_pair[l], l, false, s);
    }
}

// Start of a refinement pass: inner CG from e = 0.  Plain CG: first
// residual, z = r / 4, r.z.  Multigrid: ||r||^2, then the V-cycle of r
// with z, w = A z and the first step's alpha.
void enqueue_pass_begin(pic_ctx *c, hipStream_t s)
{
    Part pt = part_of(c);
    launch_init_red0(c->d_inst, c->t_plain, pt, s);
    if (!c->any_mg) return;
    launch_mg_down(c->d_inst, c->t_fine[0], 0, 1, 0, pt, s);
    enqueue_vcycle_mid(c, false, s);
    launch_mg_up(c->d_inst, c->t_fine[0], 0, 0, pt, s);
}

// K inner iterations; `first` when they open the pass.  Continuation chunks
// must follow an even number of iterations (plain CG: the search direction
// ping-pongs between two buffers by iteration parity; multigrid: so do the
// residual and s = A p).
void enqueue_iters(pic_ctx *c, int K, bool first, hipStream_t s)
{
    Part pt = part_of(c);
    for (int k = 0; k < K; k++) {
        launch_pupdate_Ap(c->d_inst, c->t_plain, k & 1, (first && k == 0) ? 1 : 0, pt, s);
        launch_update_red0(c->d_inst, c->t_plain, (k + 1) & 1, pt, s);
        if (!c->any_mg) continue;
        // the CG step; its reduction and stop test run in the coarse kernel
        launch_mg_down(c->d_inst, c->t_fine[0], 0, 3, k & 1, pt, s);
        enqueue_vcycle_mid(c, true, s);
        launch_mg_up(c->d_inst, c->t_fine[0], 0, (k + 1) & 1, pt, s);
    }
}

// End of a pass: phi += e, float64 residual and convergence test.
void enqueue_pass_end(pic_ctx *c, hipStream_t s)
{
    launch_phi_update(c->d_inst, c->t_l0, s);
    launch_resid64(c->d_inst, c->t_l0, 1, part_of(c), s);
}

// One refinement pass: inner preconditioned CG from e = 0 with K iterations
// (later ones return at once after the stop test), phi += e, float64 residual.
void enqueue_pass(pic_ctx *c, int K, hipStream_t s)
{
    enqueue_pass_begin(c, s);
    enqueue_iters(c, K, true, s);
    enqueue_pass_end(c, s);
}

pic_status capture_begin(pic_ctx *c)
{
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    return PIC_OK;
}

pic_status capture_end(pic_ctx *c, hipGraphExec_t *ex)
{
    hipGraph_t g = nullptr;
    *ex = nullptr;
    HIPCHK(c, hipStreamEndCapture(c->cap_stream, &g));
    hipError_t e = hipGraphInstantiate(ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, PIC_ERR_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
    return PIC_OK;
}

pic_status run_pass(pic_ctx *c, int K)
{
    if (!c->use_graphs || K > 128) {
        enqueue_pass(c, K, c->stream);
        HIPCHK(c, hipGetLastError());
        return PIC_OK;
    }
    auto it = c->outer_graphs.find(K);
    if (it == c->outer_graphs.end()) {
        pic_status st = capture_begin(c);
        if (st != PIC_OK) return st;
        enqueue_pass(c, K, c->cap_stream);
        hipGraphExec_t ex;
        st = capture_end(c, &ex);
        if (st != PIC_OK) return st;
        it = c->outer_graphs.emplace(K, ex).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    return PIC_OK;
}

// Graph of `begin + K first iterations` (first) or of K continuation
// iterations, cached by (K, first).
pic_status launch_chunk(pic_ctx *c, int K, bool first)
{
    const int key = 2 * K + (first ? 1 : 0);
    auto it = c->chunk_graphs.find(key);
    if (it == c->chunk_graphs.end()) {
        pic_status st = capture_begin(c);
        if (st != PIC_OK) return st;
        if (first) enqueue_pass_begin(c, c->cap_stream);
        enqueue_iters(c, K, first, c->cap_stream);
        hipGraphExec_t ex;
        st = capture_end(c, &ex);
        if (st != PIC_OK) return st;
        it = c->chunk_graphs.emplace(key, ex).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    return PIC_OK;
}

pic_status read_flags(pic_ctx *c, std::vector<double> &S, std::vector<int> &F)
{
    S.resize((size_t)c->n * S_NSCAL);
    F.resize((size_t)c->n * F_NFLAG);
    // one copy of the scalar and flag blocks (adjacent in the workspace) into pinned memory
    HIPCHK(c, hipMemcpyAsync(c->h_flags, c->d_S, c->flags_bytes, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    memcpy(S.data(), c->h_flags, S.size() * sizeof(double));
    memcpy(F.data(), c->h_flags + ((char *)c->d_F - (char *)c->d_S), F.size() * sizeof(int));
    for (int k = 0; k < c->n; k++) {
        const int e = F[(size_t)k * F_NFLAG + F_ERR];
        if (e) {
            c->device_error = true;
            char msg[160];
            snprintf(msg, sizeof msg, "instance %d: device error bits 0x%x%s", k, e,
                     (e & kErrVWindow) ? " (step counter outside the window of conductor potentials)" : "");
            return fail(c, PIC_ERR_STATE, msg);
        }
    }
    return PIC_OK;
}

void record_solve_info(pic_ctx *c, const std::vector<double> &S, const std::vector<int> &F)
{
    for (int k = 0; k < c->n; k++) {
        const double *s = &S[(size_t)k * S_NSCAL];
        const int *f = &F[(size_t)k * F_NFLAG];
        const double bb = s[S_BB] > 0 ? s[S_BB] : 1.0;
        pic_solve_info &si = c->in[k].last;
        si.iterations = f[F_ITER_TOT];
        si.outer = f[F_PASSES];
        si.converged = f[F_CONV];
        si.iterations_first = f[F_ITER1];
        si.relres0 = std::sqrt(s[S_RELRES0] / bb);
        si.relres = std::sqrt(s[S_RR64] / bb);
        si.unconverged_pushes = f[F_UNCONV];
        si.worst_relres = s[S_WORST];
    }
}

// Start of a solve: starting potential and the float64 residual.
void enqueue_solve_start(pic_ctx *c, int kind, const double *guess, hipStream_t s)
{
    // kind 4 keeps the time history of kind 3 (the current solution becomes
    // the previous one) and then starts from the caller's guess
    if (kind == 4) launch_extrapolate(c->d_inst, c->t_l0, 0, s);
    if (kind == 0 || kind == 2 || kind == 4) launch_set_guess(c->d_inst, c->t_l0, kind == 0 ? 0 : 2, guess, s);
    if (kind == 3) launch_extrapolate(c->d_inst, c->t_l0, c->have_prev ? 1 : 0, s);
    launch_pin_shift(c->d_inst, c->t_per, s);
    launch_resid64(c->d_inst, c->t_l0, 0, part_of(c), s);
}

constexpr int kSweepChunk = 64;       // sweeps between float64 residual tests
constexpr int kSweepKey = 1 << 20;

// `count` sweeps of the paper's iteration, then the float64 residual and its
// convergence flag (captured once per count).
pic_status run_sweep_chunk(pic_ctx *c, int count)
{
    auto enqueue = [&](hipStream_t s) {
        launch_sweeps(c->d_inst, c->t_l0, c->sweep_solver == 2 ? 1 : 0, count, s);
        launch_resid64(c->d_inst, c->t_l0, 1, part_of(c), s);
    };
    if (!c->use_graphs) {
        enqueue(c->stream);
        HIPCHK(c, hipGetLastError());
        return PIC_OK;
    }
    auto it = c->outer_graphs.find(kSweepKey + count);
    if (it == c->outer_graphs.end()) {
        pic_status st = capture_begin(c);
        if (st != PIC_OK) return st;
        enqueue(c->cap_stream);
        hipGraphExec_t ex;
        st = capture_end(c, &ex);
        if (st != PIC_OK) return st;
        it = c->outer_graphs.emplace(kSweepKey + count, ex).first;
    }
    HIPCHK(c, hipGraphLaunch(it->second, c->stream));
    return PIC_OK;
}

// The paper's own iterations to rtol: chunks of sweeps, each followed by the
// float64 residual test, until every instance converged or max_iter sweeps
// ran (Jacobi chunks are even, so a solve may run one sweep past max_iter).
// An instance's count is the sweeps run when its test first passed.
pic_status do_sweep_solve(pic_ctx *c, int kind, const double *guess)
{
    enqueue_solve_start(c, kind, guess, c->stream);
    c->have_prev = (kind == 3 || kind == 4);
    std::vector<double> S;
    std::vector<int> F;
    pic_status st = read_flags(c, S, F);
    if (st != PIC_OK) return st;
    int max_iter = 0;
    for (auto &h : c->in) max_iter = std::max(max_iter, (int)h.cfg.max_iter);
    std::vector<int> done(c->n, -1);
    int total = 0;
    auto settled = [&]() {
        bool all = true, finite = true;
        for (int k = 0; k < c->n; k++) {
            if (F[(size_t)k * F_NFLAG + F_CONV]) {
                if (done[k] < 0) done[k] = total;
            } else {
                all = false;
            }
            if (!std::isfinite(S[(size_t)k * S_NSCAL + S_RR64])) finite = false;
        }
        return all || !finite;
    };
    bool stop = settled();
    while (!stop && total < max_iter) {
        int count = std::min(kSweepChunk, max_iter - total);
        if (c->sweep_solver == 2) count += count & 1;
        if ((st = run_sweep_chunk(c, count)) != PIC_OK) return st;
        total += count;
        if ((st = read_flags(c, S, F)) != PIC_OK) return st;
        stop = settled();
    }
    launch_shift_mean(c->d_inst, c->t_per, part_of(c), c->stream);
    record_solve_info(c, S, F);
    for (int k = 0; k < c->n; k++) {
        pic_solve_info &si = c->in[k].last;
        si.iterations = si.iterations_first = done[k] >= 0 ? done[k] : total;
        si.outer = 1;
        if (!si.converged) {
            char msg[200];
            snprintf(msg, sizeof msg, "instance %d: %s stopped at relative residual %.3e after %d sweeps", k,
                     c->sweep_solver == 2 ? "Jacobi" : "Gauss-Seidel", si.relres, si.iterations);
            return fail(c, PIC_ERR_NOT_CONVERGED, msg);
        }
    }
    return PIC_OK;
}

pic_status do_solve(pic_ctx *c, int kind, const double *guess)
{
    if (c->sweep_solver) return do_sweep_solve(c, kind, guess);
    enqueue_solve_start(c, kind, guess, c->stream);
    c->have_prev = (kind == 3 || kind == 4);
    std::vector<double> S;
    std::vector<int> F;
    pic_status st = PIC_OK;
    int max_iter = 0;
    bool plain_cg = false;
    for (auto &h : c->in) {
        max_iter = std::max(max_iter, (int)h.cfg.max_iter);
        if (!h.dev.mg) plain_cg = true;
    }
    // With multigrid the first pass is queued behind the start without a
    // look at its flags (its kernels skip an instance that already
    // converged), so a solve that needs one pass costs one host round trip.
    bool have = false;
    if (plain_cg) {
        if ((st = read_flags(c, S, F)) != PIC_OK) return st;
        have = true;
    }
    for (int pass = 0; pass < 64; pass++) {
        int most = 0;
        if (have) {
            bool all = true;
            bool finite = true;
            for (int k = 0; k < c->n; k++) {
                const int *f = &F[(size_t)k * F_NFLAG];
                if (!f[F_CONV]) all = false;
                if (!std::isfinite(S[(size_t)k * S_NSCAL + S_RR64])) finite = false;
                most = std::max(most, f[F_ITER_TOT]);
            }
            if (all || !finite || most >= max_iter) break;
        }
        int &chunk = c->pass_chunk[std::min(pass, 1)];
        int K = std::max(1, std::min(std::min(chunk, 128), max_iter - most));
        if (plain_cg) {
            // Unpreconditioned CG needs long uninterrupted inner runs: continue
            // the pass's CG in graph chunks until its stop test, then update.
            K = std::min(K, 128);
            K += K & 1;
            st = launch_chunk(c, K, true);
            for (int guard = 0; st == PIC_OK && guard < (1 << 20); guard++) {
                if ((st = read_flags(c, S, F)) != PIC_OK) break;
                bool open = false;
                int tot = 0;
                for (int k = 0; k < c->n; k++) {
                    const int *f = &F[(size_t)k * F_NFLAG];
                    if (!f[F_SKIP] && !f[F_DONE]) open = true;
                    tot = std::max(tot, f[F_ITER_TOT]);
                }
                if (!open || tot >= max_iter) break;
                st = launch_chunk(c, kContinueChunk, false);
            }
            if (st != PIC_OK) return st;
            enqueue_pass_end(c, c->stream);
            HIPCHK(c, hipGetLastError());
        } else {
            st = run_pass(c, K);
        }
        if (st != PIC_OK) return st;
        st = read_flags(c, S, F);
        if (st != PIC_OK) return st;
        have = true;
        int need = 0, ran = 0;
        bool unfinished = false;
        for (int k = 0; k < c->n; k++) {
            const int *f = &F[(size_t)k * F_NFLAG];
            if (f[F_SKIP]) continue;
            ran++;
            need = std::max(need, f[F_ITER]);
            if (!f[F_DONE]) unfinished = true;
        }
        // next solve: the iterations this pass needed (passes differ: the
        // first starts far from the tolerance), doubled when it ran short;
        // a pass every instance skipped tells nothing
        if (ran) chunk = unfinished ? std::min(2 * K, 128) : std::max(1, need);
    }
    launch_shift_mean(c->d_inst, c->t_per, part_of(c), c->stream);
    record_solve_info(c, S, F);
    for (int k = 0; k < c->n; k++)
        if (!c->in[k].last.converged) {
            char msg[200];
            snprintf(msg, sizeof msg, "instance %d: solver stopped at relative residual %.3e after %d iterations",
                     k, c->in[k].last.relres, c->in[k].last.iterations);
            return fail(c, PIC_ERR_NOT_CONVERGED, msg);
        }
    return PIC_OK;
}

// field, push + deposit of both species of every instance, step + 1,
// assembly at the new time; re-binnings due after this step.
void enqueue_push(pic_ctx *c, hipStream_t s, bool timed)
{
    launch_field(c->d_inst, c->t_field, 1, s);
    const bool tm = timed && c->timing && c->nev < (int)c->ev0.size();
    if (tm) (void)hipEventRecord(c->ev0[c->nev], s);
    launch_push(c->d_push, c->t_push, true, c->unroll, c->merge, c->push_lds, s);
    if (tm) {
        (void)hipEventRecord(c->ev1[c->nev], s);
        c->nev++;
        for (auto &h : c->in) c->timed_particles += h.slots_ub[0] + h.slots_ub[1];
    }
    launch_recycle(c->d_push, c->t_recycle, s);     // before the step counter moves on
    launch_emit(c->d_see, c->t_see, c->t_see1, s);  // its charge joins rho before the assembly
    launch_tick(c->d_ctl, s);
    enqueue_assemble(c, s);
}

// The caller's stream waits for a re-binning still running on the side
// stream (no host wait).
void join_bin(pic_ctx *c)
{
    if (!c->bin_pending) return;
    (void)hipStreamWaitEvent(c->stream, c->ev_bin_done, 0);
    c->bin_pending = false;
}

int sorts_due(pic_ctx *c, long long step_after)
{
    int mask = 0;
    for (int sp = 0; sp < 2; sp++) {
        const int K = c->in[0].cfg.sort_interval[sp];
        if (K > 0 && step_after % K == 0) mask |= 1 << sp;
    }
    return mask;
}

// side: a re-binning that falls due may run on the side stream until the
// next push (pic_step's loop, whose solve in between touches no particle).
pic_status do_push(pic_ctx *c, bool side = false)
{
    pic_status st = ensure_vwindow(c, c->step + 1, 1);
    if (st != PIC_OK) return st;
    join_bin(c);
    enqueue_push(c, c->stream, true);
    c->step++;
    const int mask = sorts_due(c, c->step);
    if (mask && side) {
        if (!c->bin_stream) {
            HIPCHK(c, hipStreamCreateWithFlags(&c->bin_stream, hipStreamNonBlocking));
            HIPCHK(c, hipEventCreateWithFlags(&c->ev_bin_go, hipEventDisableTiming));
            HIPCHK(c, hipEventCreateWithFlags(&c->ev_bin_done, hipEventDisableTiming));
        }
        HIPCHK(c, hipEventRecord(c->ev_bin_go, c->stream));
        HIPCHK(c, hipStreamWaitEvent(c->bin_stream, c->ev_bin_go, 0));
        enqueue_bin(c, mask, c->bin_stream);
        HIPCHK(c, hipEventRecord(c->ev_bin_done, c->bin_stream));
        c->bin_pending = true;
    } else if (mask) {
        enqueue_bin(c, mask, c->stream);
    }
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status check(pic_ctx *c)
{
    if (!c || !c->d_inst) return fail(c, PIC_ERR_STATE, "not initialised");
    if (c->device_error) return PIC_ERR_STATE;     // the message of the first report stays
    join_bin(c);
    return PIC_OK;
}

pic_status init_instance(pic_ctx *c, int k, const pic_config *cfg, const pic_buffers *buf)
{
    InstHost &h = c->in[k];
    const int64_t cap[2] = {buf->sp[0].capacity, buf->sp[1].capacity};
    h.cfg = *cfg;
    h.cell_cond.assign(cfg->cell_cond, cfg->cell_cond + (size_t)cfg->nx * cfg->ny);
    h.cfg.cell_cond = h.cell_cond.data();
    for (auto v8 : h.cell_cond)
        if (v8 >= PIC_MAX_COND) return fail(c, PIC_ERR_ARG, "cell conductor id above 7");
    if (!node_map(&h.cfg, h.node_cond))
        return fail(c, PIC_ERR_ARG, "two different conductors meet at a node");
    h.L = make_layout(&h.cfg, cap);
    const Layout &L = h.L;
    h.buf = *buf;
    h.g = Geom{L.nx, L.ny, L.NX, L.NY, L.px, L.py};
    for (int s = 0; s < 2; s++) {
        h.loaded[s] = buf->sp[s].count;
        h.slots_ub[s] = buf->sp[s].count;
    }
    // emitted electrons are appended to species 0, up to its capacity
    if (see_on(cfg)) h.slots_ub[0] = buf->sp[0].capacity;
    // masks of every level: level 0 = Dirichlet nodes (plus node 0 pinned on a
    // fully periodic grid); coarse node fixed iff its coincident fine node is
    h.fixh.assign(L.nlev, {});
    h.fixh[0].resize((size_t)L.NX * L.NY);
    for (size_t q = 0; q < h.fixh[0].size(); q++) h.fixh[0][q] = h.node_cond[q] ? 1 : 0;
    if (L.px && L.py) h.fixh[0][0] = 1;
    for (int l = 1; l < L.nlev; l++) {
        const int NXc = L.NXl[l], NYc = L.NYl[l], NYf = L.NYl[l - 1];
        h.fixh[l].resize((size_t)NXc * NYc);
        for (int I = 0; I < NXc; I++)
            for (int J = 0; J < NYc; J++)
                h.fixh[l][(size_t)I * NYc + J] = h.fixh[l - 1][(size_t)(2 * I) * NYf + 2 * J];
    }
    h.dense = L.dense_n && coarse_inverse(h.fixh[L.nlev - 1], L.NXl[L.nlev - 1], L.NYl[L.nlev - 1], h.ainvh);
    hipStream_t s = c->stream;
    if (h.dense)
        HIPCHK(c, hipMemcpyAsync(h.d_ainv, h.ainvh.data(), h.ainvh.size() * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(h.d_cell_cond, h.cell_cond.data(), h.cell_cond.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(h.d_node_cond, h.node_cond.data(), h.node_cond.size(), hipMemcpyHostToDevice, s));
    for (int l = 0; l < L.nlev; l++)
        HIPCHK(c, hipMemcpyAsync(h.d_fix[l], h.fixh[l].data(), h.fixh[l].size(), hipMemcpyHostToDevice, s));
    // device descriptor
    Inst &d = h.dev;
    memset(&d, 0, sizeof d);
    d.g = h.g;
    d.nlev = L.nlev;
    d.lg = L.mg ? L.lg : 0;
    d.mg = L.mg ? 1 : 0;
    for (int l = 0; l < L.nlev; l++) {
        d.lev[l].NX = L.NXl[l];
        d.lev[l].NY = L.NYl[l];
        d.lev[l].u = h.d_u[l];
        d.lev[l].uo = h.d_uo[l];
        d.lev[l].g = h.d_g[l];
        d.lev[l].fix = h.d_fix[l];
    }
    d.z = h.d_u[0];
    d.node_cond = h.d_node_cond;
    d.cell_cond = h.d_cell_cond;
    d.phi = buf->phi;
    d.b = buf->b;
    d.phi_prev = h.d_phi_prev;
    d.phi2 = h.d_phi2;
    d.rho[0] = reinterpret_cast<unsigned long long *>(buf->rho[0]);
    d.rho[1] = reinterpret_cast<unsigned long long *>(buf->rho[1]);
    d.e = h.d_e;
    d.p[0] = h.d_p[0];
    d.p[1] = h.d_p[1];
    d.q = h.d_q;
    d.cg_r1 = h.d_cg_r1;
    d.cg_s[0] = h.d_cg_s[0];
    d.cg_s[1] = h.d_cg_s[1];
    d.cg_w = h.d_cg_w;
    d.E4 = h.d_E4;
    d.S = c->d_S + (size_t)k * S_NSCAL;
    d.F = c->d_F + (size_t)k * F_NFLAG;
    d.surf = h.d_surf;
    d.qcharge = std::ldexp(h.cfg.weight, -32);
    d.charge_mode = h.cfg.charge_mode;
    d.charge_row = h.cfg.charge_row;
    d.sjl = h.cfg.static_j_lo;
    d.sjh = h.cfg.static_j_hi;
    d.sden = h.cfg.static_density;
    d.rtol = h.cfg.rtol;
    d.eta_min = d.mg ? 5e-7 : 1e-5;
    if (L.mg) {
        CoarseArgs &ca = d.coarse;
        ca.nlev = L.nlev - L.lg;
        int off = 0;
        for (int q = 0; q < ca.nlev; q++) {
            const int l = L.lg + q;
            const int nn = L.NXl[l] * L.NYl[l];
            ca.NX[q] = L.NXl[l];
            ca.NY[q] = L.NYl[l];
            ca.off_u[q] = off;
            off += (nn * 4 + 15) & ~15;
            ca.off_g[q] = off;
            off += (nn * 4 + 15) & ~15;
            ca.off_f[q] = off;
            off += (nn + 15) & ~15;
            ca.fix[q] = h.d_fix[l];
        }
        ca.off_s = off;
        off += (L.NXl[L.lg] * L.NYl[L.lg] * 4 + 15) & ~15;
        ca.off_p = off;
        if (h.dense) off += (kCoarseWaves * L.dense_n * 4 + 15) & ~15;
        ca.lds_bytes = off;
        ca.u_top = h.d_u[L.lg];
        ca.g_top = h.d_g[L.lg];
        ca.px = L.px;
        ca.py = L.py;
        const int last = ca.nlev - 1;
        ca.sweeps = std::min(64, std::max(2, std::max(ca.NX[last], ca.NY[last])));
        ca.ainv = h.dense ? h.d_ainv : nullptr;
        ca.dense_n = h.dense ? L.dense_n : 0;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_inst + k, &d, sizeof d, hipMemcpyHostToDevice, s));
    // particle kernels' arguments (both storage sets; info[7] selects)
    for (int sp = 0; sp < 2; sp++) {
        PushArgs a;
        memset(&a, 0, sizeof a);
        a.g = h.g;
        a.TX = L.TX;
        a.TY = L.TY;
        a.lx = L.lx;
        a.ly = L.ly;
        a.tiles_y = L.tiles_y;
        a.H = L.H;
        a.WX = L.TX + 2 * L.H;
        a.WY = L.TY + 2 * L.H;
        a.cell_cond = h.d_cell_cond;
        a.E4 = h.d_E4;
        for (int q = 0; q < 2; q++) {
            a.cell[q] = buf->sp[sp].cell[q];
            a.ox[q] = buf->sp[sp].ox[q];
            a.oy[q] = buf->sp[sp].oy[q];
            a.vx[q] = buf->sp[sp].vx[q];
            a.vy[q] = buf->sp[sp].vy[q];
        }
        a.table = h.d_table[sp];
        a.info = h.d_info[sp];
        a.rho = reinterpret_cast<unsigned long long *>(buf->rho[sp]);
        a.qdt = (float)(h.cfg.alpha[sp] * h.cfg.dt);
        a.dtf = (float)h.cfg.dt;
        a.hq = (float)(0.5 * h.cfg.alpha[sp] * h.cfg.dt);
        a.box_i_top = h.cfg.box_i_top;
        a.box_j_lo = h.cfg.box_j_lo;
        a.box_j_hi = h.cfg.box_j_hi;
        a.species = sp;
        a.inst = k;
        a.tally = h.d_tally + sp * kNClass;
        a.surf = (h.cfg.charge_mode == 2 && sp == 1) ? h.d_surf : nullptr;
        a.iad = (sp == 1 && h.cfg.box_i_top < h.cfg.nx) ? h.d_iad : nullptr;
        a.recycle_rows = sp == 1 ? h.cfg.recycle_rows : 0;
        a.recycle_key[0] = h.cfg.recycle_key[0];
        a.recycle_key[1] = h.cfg.recycle_key[1];
        a.recycle_vth = h.cfg.recycle_vth;
        a.log.rec = h.cfg.hitlog_capacity > 0 ? h.d_hits : nullptr;
        a.log.count = h.d_misc + 1;
        a.log.capacity = std::max<int64_t>(h.cfg.hitlog_capacity, 1);
        a.log.species_mask = h.cfg.hitlog_species_mask;
        a.step = c->d_ctl;
        a.fallbacks = h.d_misc + 0;
        HIPCHK(c, hipMemcpyAsync(c->d_push + 2 * k + sp, &a, sizeof a, hipMemcpyHostToDevice, s));
        BinArgs b;
        memset(&b, 0, sizeof b);
        b.nx = L.nx;
        b.ny = L.ny;
        b.lx = L.lx;
        b.ly = L.ly;
        b.tiles_y = L.tiles_y;
        b.ntiles = L.ntiles;
        b.chunk = L.chunk;
        b.bad = h.d_misc + 2;
        for (int q = 0; q < 2; q++) {
            b.cell[q] = buf->sp[sp].cell[q];
            b.ox[q] = buf->sp[sp].ox[q];
            b.oy[q] = buf->sp[sp].oy[q];
            b.vx[q] = buf->sp[sp].vx[q];
            b.vy[q] = buf->sp[sp].vy[q];
        }
        b.counts = h.d_counts[sp];
        b.offsets = h.d_offsets[sp];
        b.cursor = h.d_cursor[sp];
        b.boff = h.d_boff[sp];
        b.table = h.d_table[sp];
        b.info = h.d_info[sp];
        HIPCHK(c, hipMemcpyAsync(c->d_bin + 2 * k + sp, &b, sizeof b, hipMemcpyHostToDevice, s));
        long long info[8] = {0, 0, buf->sp[sp].count, 0, buf->sp[sp].count, 0, 0, 0};
        HIPCHK(c, hipMemcpyAsync(h.d_info[sp], info, sizeof info, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));   // the small host structs above go out of scope
    }
    {
        SeeArgs e;
        memset(&e, 0, sizeof e);
        e.g = h.g;
        e.rec = h.d_hits;
        e.log_count = h.d_misc + 1;
        e.log_capacity = std::max<int64_t>(h.cfg.hitlog_capacity, 1);
        e.misc = h.d_misc + 8;
        for (int sp = 0; sp < 2; sp++)
            e.thresh[sp] = (unsigned)std::floor(h.cfg.see_yield[sp] * 16777216.0);
        e.vth = h.cfg.see_vth;
        e.key[0] = h.cfg.see_key[0];
        e.key[1] = h.cfg.see_key[1];
        for (int q = 0; q < 2; q++) {
            e.cell[q] = buf->sp[0].cell[q];
            e.ox[q] = buf->sp[0].ox[q];
            e.oy[q] = buf->sp[0].oy[q];
            e.vx[q] = buf->sp[0].vx[q];
            e.vy[q] = buf->sp[0].vy[q];
        }
        e.info = h.d_info[0];
        e.table = h.d_table[0];
        e.capacity = buf->sp[0].capacity;
        e.chunk = L.chunk;
        e.rho = reinterpret_cast<unsigned long long *>(buf->rho[0]);
        HIPCHK(c, hipMemcpyAsync(c->d_see + k, &e, sizeof e, hipMemcpyHostToDevice, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    HIPCHK(c, hipMemsetAsync(h.d_tally, 0, sizeof(unsigned long long) * 2 * kNClass, s));
    HIPCHK(c, hipMemsetAsync(h.d_surf, 0, sizeof(unsigned long long) * (L.ny + 1), s));
    HIPCHK(c, hipMemsetAsync(h.d_misc, 0, sizeof(unsigned long long) * 16, s));
    HIPCHK(c, hipMemsetAsync(h.d_iad, 0, sizeof(unsigned long long) * kIadBins, s));
    HIPCHK(c, hipMemsetAsync(h.d_e, 0, sizeof(float) * (size_t)L.NX * L.NY, s));
    HIPCHK(c, hipMemsetAsync(h.d_p[0], 0, sizeof(float) * (size_t)L.NX * L.NY, s));
    HIPCHK(c, hipMemsetAsync(h.d_p[1], 0, sizeof(float) * (size_t)L.NX * L.NY, s));
    if (L.mg) {
        for (float *b : {h.d_cg_r1, h.d_cg_s[0], h.d_cg_s[1], h.d_cg_w})
            HIPCHK(c, hipMemsetAsync(b, 0, sizeof(float) * (size_t)L.NX * L.NY, s));
    }
    HIPCHK(c, hipMemsetAsync(h.d_counts[0], 0, sizeof(unsigned) * L.ntiles, s));
    HIPCHK(c, hipMemsetAsync(h.d_counts[1], 0, sizeof(unsigned) * L.ntiles, s));
    HIPCHK(c, hipMemsetAsync(buf->phi, 0, sizeof(double) * (size_t)L.NX * L.NY, s));
    return PIC_OK;
}

void build_tabs(pic_ctx *c)
{
    c->t_l0 = c->t_field = c->t_per = c->t_coarse = c->t_push = c->t_rewind = c->t_plain = c->t_recycle = Tab{};
    c->t_see = c->t_see1 = Tab{};
    for (int l = 0; l < kMaxLev; l++) c->t_fine[l] = c->t_pair[l] = Tab{};
    c->maxlg = 0;
    c->coarse_lds = 0;
    c->any_mg = 0;
    c->push_lds = 0;
    for (int k = 0; k < c->n; k++) {
        const InstHost &h = c->in[k];
        const Layout &L = h.L;
        tab_add_grid(c->t_l0, k, L.NX, L.NY);
        tab_add_grid(c->t_field, k, std::max(L.NX, L.nx), std::max(L.NY, L.ny));
        if (L.px && L.py) tab_add_grid(c->t_per, k, L.NX, L.NY);
        if (!L.mg) tab_add_grid(c->t_plain, k, L.NX, L.NY);
        if (L.mg) {
            c->any_mg = 1;
            c->maxlg = std::max(c->maxlg, L.lg);
            // level 0 alone (it carries the CG step); levels 1 .. lg-1 in pairs
            // (1, 2), (3, 4), ..., a last odd one alone
            for (int l = 0; l < L.lg; l++) {
                const bool pair = c->pair_levels && l >= 1 && (l & 1) && l + 1 < L.lg;
                const int lt = pair ? l + 1 : l;
                const int tx = (L.NXl[lt] + kMgTileHost - 1) / kMgTileHost;
                const int ty = (L.NYl[lt] + kMgTileHost - 1) / kMgTileHost;
                Tab &tb = pair ? c->t_pair[l] : c->t_fine[l];
                const int q = tb.n;
                tab_add(tb, k, tx * ty);
                tb.bx[q] = ty;
                if (pair) l++;
            }
            tab_add(c->t_coarse, k, 1);
            c->coarse_lds = std::max(c->coarse_lds, h.dev.coarse.lds_bytes);
        }
        for (int s = 0; s < 2; s++) {
            tab_add(c->t_push, 2 * k + s, (int)L.max_blocks[s]);
            tab_add(c->t_rewind, 2 * k + s, (int)((h.slots_ub[s] + 255) / 256));
            if (s == 1 && h.cfg.recycle_rows > 0)
                tab_add(c->t_recycle, 2 * k + s, (int)std::max<long long>(1, (h.slots_ub[s] + 255) / 256));
        }
        c->push_lds = std::max(c->push_lds, push_lds_bytes(L.TX, L.TY, L.H));
        if (see_on(&h.cfg)) {
            tab_add(c->t_see, k, kEmitBlocks);
            tab_add(c->t_see1, k, 1);
        }
    }
    c->unroll = c->in[0].L.unroll;
    c->merge = c->in[0].L.merge;
}

pic_status batch_init(int n, const pic_config *cfgs, const pic_buffers *bufs, void *ws, size_t wsb,
                      void *stream, pic_ctx **out)
{
    if (!out) return PIC_ERR_ARG;
    *out = nullptr;
    pic_ctx *c = new (std::nothrow) pic_ctx();
    if (!c) return PIC_ERR_ARG;
    *out = c;
    if (n < 1 || n > kMaxInst) return fail(c, PIC_ERR_ARG, "instance count must be 1..16");
    if (!cfgs || !bufs) return fail(c, PIC_ERR_ARG, "null configurations or buffers");
    if (!ws) return fail(c, PIC_ERR_ARG, "missing workspace");
    if (reinterpret_cast<uintptr_t>(ws) & 255) return fail(c, PIC_ERR_ARG, "workspace must be 256-byte aligned");
    std::vector<int64_t> caps(2 * n);
    for (int k = 0; k < n; k++) {
        const pic_buffers *b = &bufs[k];
        caps[2 * k] = b->sp[0].capacity;
        caps[2 * k + 1] = b->sp[1].capacity;
        std::string v = validate(&cfgs[k], &caps[2 * k]);
        if (!v.empty()) return fail(c, validate_status(v), "instance " + std::to_string(k) + ": " + v);
        {
            // leapfrog stability of the electron plasma oscillation at the loaded
            // mean density n (omega_pe^2 = |alpha_e| n in the units of Sec. II):
            // omega_pe dt must stay below 2
            long long plasma = 0;
            for (long long q = 0; q < (long long)cfgs[k].nx * cfgs[k].ny; q++) plasma += cfgs[k].cell_cond[q] == 0;
            const double dens = plasma > 0 ? cfgs[k].weight * (double)b->sp[0].count / (double)plasma : 0.0;
            const double wdt = cfgs[k].dt * std::sqrt(std::fabs(cfgs[k].alpha[0]) * dens);
            if (!(wdt < 2.0)) {
                char msg[160];
                snprintf(msg, sizeof msg, "instance %d: omega_pe dt = %.3g at the loaded mean density: the leapfrog "
                         "is unstable (needs < 2)", k, wdt);
                return fail(c, PIC_ERR_CFL, msg);
            }
        }
        for (int s = 0; s < 2; s++) {
            if (b->sp[s].count < 0 || b->sp[s].count > b->sp[s].capacity)
                return fail(c, PIC_ERR_CAPACITY, "particle count exceeds capacity");
            for (int q = 0; q < 2; q++)
                if (b->sp[s].capacity > 0 &&
                    (!b->sp[s].cell[q] || !b->sp[s].ox[q] || !b->sp[s].oy[q] || !b->sp[s].vx[q] || !b->sp[s].vy[q]))
                    return fail(c, PIC_ERR_ARG, "missing particle buffer");
            if (!b->rho[s]) return fail(c, PIC_ERR_ARG, "missing rho buffer");
        }
        if (!b->phi || !b->b) return fail(c, PIC_ERR_ARG, "missing phi or b");
        const int us = cfgs[k].push_unroll, ms = cfgs[k].push_merge;
        if (k > 0 && (us != cfgs[0].push_unroll || ms != cfgs[0].push_merge))
            return fail(c, PIC_ERR_ARG, "all instances of a batch use one push variant");
    }
    const size_t need = carve_all(nullptr, n, cfgs, caps.data(), nullptr);
    if (wsb < need) return fail(c, PIC_ERR_ARG, "workspace too small");
    c->n = n;
    c->in.resize(n);
    c->stream = reinterpret_cast<hipStream_t>(stream);
    carve_all(c, n, cfgs, caps.data(), reinterpret_cast<char *>(ws));
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemsetAsync(c->d_S, 0, sizeof(double) * n * S_NSCAL, s));
    HIPCHK(c, hipMemsetAsync(c->d_F, 0, sizeof(int) * n * F_NFLAG, s));
    c->flags_bytes = (size_t)((char *)(c->d_F + (size_t)n * F_NFLAG) - (char *)c->d_S);
    HIPCHK(c, hipHostMalloc((void **)&c->h_flags, c->flags_bytes, hipHostMallocDefault));
    for (int k = 0; k < n; k++) {
        pic_status st = init_instance(c, k, &cfgs[k], &bufs[k]);
        if (st != PIC_OK) return st;
    }
    for (int k = 0; k < n; k++) {
        const int sk = cfgs[k].solver >= 2 ? cfgs[k].solver : 0;
        if (k > 0 && sk != c->sweep_solver)
            return fail(c, PIC_ERR_ARG, "a batch mixes no CG and sweep solvers, nor Jacobi and Gauss-Seidel");
        c->sweep_solver = sk;
    }
    build_tabs(c);
    c->step = 0;
    pic_status st = upload_vwindow(c, 0);
    if (st != PIC_OK) return st;
    enqueue_bin(c, 3, s);
    c->ev0.resize(kMaxTiming);
    c->ev1.resize(kMaxTiming);
    for (int k = 0; k < kMaxTiming; k++) {
        HIPCHK(c, hipEventCreate(&c->ev0[k]));
        HIPCHK(c, hipEventCreate(&c->ev1[k]));
    }
    enqueue_deposit(c, s);
    HIPCHK(c, hipGetLastError());
    std::vector<unsigned long long> bad(n);
    for (int k = 0; k < n; k++)
        HIPCHK(c, hipMemcpyAsync(&bad[k], c->in[k].d_misc + 2, 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int k = 0; k < n; k++)
        if (bad[k]) return fail(c, PIC_ERR_ARG, "particles with cell codes outside the grid");
    for (auto &h : c->in) {
        h.fixh.clear();
        h.ainvh = std::vector<float>();
    }
    return PIC_OK;
}

// Captured graph of P whole steps (fixed solver schedule: `passes` passes of
// K iterations with per-instance early exit) ending with the re-binnings in
// sort_mask.
pic_status step_graph(pic_ctx *c, int P, int passes, int K, int K2, int sort_mask, hipGraphExec_t *ex)
{
    const long long key = ((long long)P << 32) | ((long long)passes << 28) | ((long long)K << 20) |
                          ((long long)K2 << 12) | sort_mask;
    auto it = c->step_graphs.find(key);
    if (it != c->step_graphs.end()) {
        *ex = it->second;
        return PIC_OK;
    }
    pic_status st = capture_begin(c);
    if (st != PIC_OK) return st;
    hipStream_t s = c->cap_stream;
    for (int k = 0; k < P; k++) {
        enqueue_solve_start(c, 3, nullptr, s);
        for (int q = 0; q < passes; q++) enqueue_pass(c, q == 0 ? K : K2, s);
        launch_shift_mean(c->d_inst, c->t_per, part_of(c), s);
        enqueue_push(c, s, false);
    }
    if (sort_mask) enqueue_bin(c, sort_mask, s);
    st = capture_end(c, ex);
    if (st != PIC_OK) return st;
    c->step_graphs.emplace(key, *ex);
    return PIC_OK;
}

} // namespace

extern "C" {

const char *pic_version(void) { return "pic-gfx950 1.1"; }

const char *pic_last_error(const pic_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

pic_status pic_node_map(pic_ctx *ctx, int32_t i, const uint8_t **node_cond, uint8_t *host_copy,
                        int32_t *NX, int32_t *NY)
{
    if (!ctx) return PIC_ERR_ARG;
    if (i < 0 || i >= ctx->n) return fail(ctx, PIC_ERR_ARG, "pic_node_map: bad instance");
    const InstHost &h = ctx->in[i];
    if (node_cond) *node_cond = h.d_node_cond;
    if (host_copy) std::memcpy(host_copy, h.node_cond.data(), h.node_cond.size());
    if (NX) *NX = h.g.NX;
    if (NY) *NY = h.g.NY;
    return PIC_OK;
}

pic_status pic_batch_workspace_size(int32_t n, const pic_config *cfgs, const int64_t *capacity, size_t *bytes)
{
    if (n < 1 || n > kMaxInst || !cfgs || !capacity || !bytes) return PIC_ERR_ARG;
    for (int k = 0; k < n; k++) {
        std::string v = validate(&cfgs[k], capacity + 2 * k);
        if (!v.empty()) return validate_status(v);
    }
    *bytes = carve_all(nullptr, n, cfgs, capacity, nullptr);
    return PIC_OK;
}

pic_status pic_workspace_size(const pic_config *cfg, const int64_t *capacity, size_t *bytes)
{
    return pic_batch_workspace_size(1, cfg, capacity, bytes);
}

pic_status pic_init(const pic_config *cfg, const pic_buffers *buf, void *stream, pic_ctx **out)
{
    if (!buf) {
        if (out) *out = nullptr;
        return PIC_ERR_ARG;
    }
    return batch_init(1, cfg, buf, buf->workspace, buf->workspace_bytes, stream, out);
}

pic_status pic_batch_init(int32_t n, const pic_config *cfgs, const pic_buffers *bufs, void *workspace,
                          size_t workspace_bytes, void *stream, pic_ctx **out)
{
    return batch_init(n, cfgs, bufs, workspace, workspace_bytes, stream, out);
}

pic_status pic_deposit(pic_ctx *c)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    pic_status st = ensure_vwindow(c, c->step, 0);
    if (st != PIC_OK) return st;
    enqueue_deposit(c, c->stream);
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status pic_solve(pic_ctx *c, int32_t guess_kind, const double *guess, pic_solve_info *info)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (guess_kind < 0 || guess_kind > 4 || ((guess_kind == 2 || guess_kind == 4) && (!guess || c->n != 1)))
        return fail(c, PIC_ERR_ARG, "guess_kind must be 0, 1, 2 or 4 (one instance, with a guess array) or 3");
    pic_status st = do_solve(c, guess_kind, guess);
    if (info) *info = c->in[0].last;
    return st;
}

pic_status pic_rewind(pic_ctx *c)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    launch_field(c->d_inst, c->t_field, 0, c->stream);
    launch_rewind(c->d_push, c->t_rewind, c->stream);
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status pic_push(pic_ctx *c)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    return do_push(c);
}

pic_status pic_step(pic_ctx *c, int32_t nsteps)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (nsteps < 0) return fail(c, PIC_ERR_ARG, "nsteps < 0");
    for (int k = 0; k < nsteps; k++) {
        pic_status st = do_solve(c, c->in[0].cfg.warm_start == 1 ? 3 : 1, nullptr);
        if (st == PIC_OK) st = do_push(c, true);
        if (st != PIC_OK) {
            join_bin(c);
            return st;
        }
    }
    // work the caller queues next (particle views included) follows the re-binning
    join_bin(c);
    return PIC_OK;
}

pic_status pic_batch_step(pic_ctx *c, int32_t nsteps, int32_t passes, int32_t iters, int32_t iters_later)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (iters_later == 0) iters_later = iters;
    if (nsteps < 0 || passes < 1 || passes > 8 || iters < 1 || iters > 128 || iters_later < 1 || iters_later > 128)
        return fail(c, PIC_ERR_ARG, "nsteps >= 0, passes in 1..8, iters and iters_later in 1..128");
    if (c->sweep_solver) return fail(c, PIC_ERR_ARG, "pic_batch_step needs the CG solvers (solver 0 or 1)");
    if (nsteps == 0) return PIC_OK;
    // pushes made so far with an unconverged potential (sticky device count)
    std::vector<double> S;
    std::vector<int> F;
    pic_status st = read_flags(c, S, F);
    if (st != PIC_OK) return st;
    std::vector<int> unconv0(c->n);
    for (int k = 0; k < c->n; k++) unconv0[k] = F[(size_t)k * F_NFLAG + F_UNCONV];
    if (!c->have_prev) {
        // the captured schedule extrapolates from two earlier solutions
        st = pic_step(c, 1);
        if (st != PIC_OK && st != PIC_ERR_NOT_CONVERGED) return st;
        nsteps--;
    }
    const int P = c->in[0].cfg.sort_interval[0] > 0 ? c->in[0].cfg.sort_interval[0] : 8;
    while (nsteps > 0) {
        // a graph covers at most one re-binning period and never more steps
        // than the device window of conductor potentials holds
        const int len = (int)std::min<long long>(std::min<long long>(nsteps, P - (c->step % P)),
                                                 kVWindow - 2);
        st = ensure_vwindow(c, c->step, len + 1);
        if (st != PIC_OK) return st;
        const int mask = sorts_due(c, c->step + len);
        hipGraphExec_t ex;
        st = step_graph(c, len, passes, iters, iters_later, mask, &ex);
        if (st != PIC_OK) return st;
        HIPCHK(c, hipGraphLaunch(ex, c->stream));
        c->step += len;
        nsteps -= len;
    }
    st = read_flags(c, S, F);
    if (st != PIC_OK) return st;
    record_solve_info(c, S, F);
    for (int k = 0; k < c->n; k++) {
        const int d = F[(size_t)k * F_NFLAG + F_UNCONV] - unconv0[k];
        if (d > 0) {
            char msg[200];
            snprintf(msg, sizeof msg, "instance %d: %d of the steps pushed a potential above rtol "
                     "(largest relative residual so far %.3e)", k, d, S[(size_t)k * S_NSCAL + S_WORST]);
            return fail(c, PIC_ERR_NOT_CONVERGED, msg);
        }
    }
    return PIC_OK;
}

pic_status pic_inject_fault(pic_ctx *c, int32_t what)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (what != 1) return fail(c, PIC_ERR_ARG, "pic_inject_fault: what must be 1");
    // the device step counter jumps past the window of conductor potentials,
    // as a runtime that lost track of it would leave it
    for (int k = 0; k < kVWindow; k++) launch_tick(c->d_ctl, c->stream);
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status pic_tune(pic_ctx *c, int32_t push_unroll, int32_t push_merge, int32_t sort_e, int32_t sort_i)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (push_unroll != 1 && push_unroll != 2 && push_unroll != 4)
        return fail(c, PIC_ERR_ARG, "push_unroll must be 1, 2 or 4");
    if (push_merge != 0 && push_merge != 2 && push_merge != 4)
        return fail(c, PIC_ERR_ARG, "push_merge must be 0, 2 or 4");
    if (sort_e < 0 || sort_i < 0 || sort_e > 1 << 20 || sort_i > 1 << 20)
        return fail(c, PIC_ERR_ARG, "sort intervals must be in 0 .. 2^20");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->unroll = push_unroll;
    c->merge = push_merge;
    for (auto &h : c->in) {
        h.cfg.push_unroll = push_unroll;
        h.cfg.push_merge = push_merge;
        h.cfg.sort_interval[0] = sort_e;
        h.cfg.sort_interval[1] = sort_i;
        h.L.unroll = push_unroll;
        h.L.merge = push_merge;
    }
    // captured steps embed the push variant and the re-binning points
    for (auto &kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
    c->step_graphs.clear();
    return PIC_OK;
}

pic_status pic_set_level_pairs(pic_ctx *c, int32_t on)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (on != 0 && on != 1) return fail(c, PIC_ERR_ARG, "on must be 0 or 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->pair_levels = on;
    build_tabs(c);
    // every captured graph embeds the V-cycle's launches
    for (auto &kv : c->outer_graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : c->chunk_graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
    c->outer_graphs.clear();
    c->chunk_graphs.clear();
    c->step_graphs.clear();
    return PIC_OK;
}

pic_status pic_sort(pic_ctx *c, int32_t species)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (species < 0 || species > 1) return fail(c, PIC_ERR_ARG, "species must be 0 or 1");
    enqueue_bin(c, 1 << species, c->stream);
    HIPCHK(c, hipGetLastError());
    return PIC_OK;
}

pic_status pic_batch_diagnostics(pic_ctx *c, int32_t i, pic_diag *out)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (!out || i < 0 || i >= c->n) return fail(c, PIC_ERR_ARG, "bad instance or output");
    InstHost &h = c->in[i];
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemsetAsync(h.d_misc + 4, 0, 2 * sizeof(unsigned long long), s));
    for (int sp = 0; sp < 2; sp++)
        launch_rho_sum(reinterpret_cast<const unsigned long long *>(h.buf.rho[sp]),
                       (long long)h.g.NX * h.g.NY, h.d_misc + 4 + sp, s);
    for (int sp = 0; sp < 2; sp++)
        launch_kinetic(c->d_push, 2 * i + sp, h.d_diag, h.d_diag + kDiagBlocks + sp, s);
    launch_field_energy(c->d_inst, i, h.d_diag, h.d_diag + kDiagBlocks + 2, s);
    unsigned long long tally[2 * kNClass], misc[16], iad[kIadBins];
    double dsum[4];
    std::vector<unsigned long long> surf(h.L.ny + 1);
    HIPCHK(c, hipMemcpyAsync(tally, h.d_tally, sizeof tally, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(iad, h.d_iad, sizeof iad, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(dsum, h.d_diag + kDiagBlocks, sizeof dsum, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(misc, h.d_misc, sizeof misc, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(surf.data(), h.d_surf, surf.size() * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    {
        // device error bits and the sticky unconverged-push count
        std::vector<double> S;
        std::vector<int> F;
        pic_status st = read_flags(c, S, F);
        if (st != PIC_OK) return st;
        h.last.unconverged_pushes = F[(size_t)i * F_NFLAG + F_UNCONV];
        h.last.worst_relres = S[(size_t)i * S_NSCAL + S_WORST];
    }
    memset(out, 0, sizeof *out);
    out->step = c->step;
    out->t = c->step * h.cfg.dt;
    for (int sp = 0; sp < 2; sp++) {
        long long lost = 0;
        // recycled ions (classes 0..7 of species 1) come back in the same push
        const bool recycled = sp == 1 && h.cfg.recycle_rows > 0;
        for (int k = 0; k < kNClass; k++) {
            out->tally[sp][k] = (int64_t)tally[sp * kNClass + k];
            if (!recycled || k == kNClass - 1) lost += (long long)tally[sp * kNClass + k];
        }
        out->loaded[sp] = h.loaded[sp];
        out->alive[sp] = h.loaded[sp] - lost + (sp == 0 ? (long long)misc[10] : 0);
        out->charge[sp] = (int64_t)misc[4 + sp];
    }
    long long sh = 0;
    for (auto v8 : surf) sh += (long long)v8;
    out->surf_hits = sh;
    out->hits_logged = (int64_t)misc[1];
    out->deposit_fallbacks = (int64_t)misc[0];
    out->last_solve = h.last;
    for (int sp = 0; sp < 2; sp++)
        out->kinetic[sp] = 0.5 * h.cfg.weight * dsum[sp] / std::fabs(h.cfg.alpha[sp]);
    out->field_energy = dsum[2];
    for (int k = 0; k < kIadBins; k++) out->iad[k] = (int64_t)iad[k];
    out->see_emitted = (int64_t)misc[10];
    out->see_dropped = (int64_t)misc[11];
    return PIC_OK;
}

pic_status pic_diagnostics(pic_ctx *c, pic_diag *out) { return pic_batch_diagnostics(c, 0, out); }

pic_status pic_batch_particles(pic_ctx *c, int32_t i, int32_t species, int32_t *set, int64_t *slots)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (i < 0 || i >= c->n || species < 0 || species > 1) return fail(c, PIC_ERR_ARG, "bad instance or species");
    long long info[8];
    HIPCHK(c, hipMemcpyAsync(info, c->in[i].d_info[species], sizeof info, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (set) *set = (int32_t)info[7];
    if (slots) *slots = info[2 + info[7]];
    return PIC_OK;
}

pic_status pic_particles(pic_ctx *c, int32_t species, int32_t *set, int64_t *slots)
{
    return pic_batch_particles(c, 0, species, set, slots);
}

pic_status pic_read_hits(pic_ctx *c, pic_hit *out, int64_t max, int64_t *n)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (!out || !n || max < 0) return fail(c, PIC_ERR_ARG, "bad output");
    *n = 0;
    InstHost &h = c->in[0];
    if (h.cfg.hitlog_capacity <= 0) return PIC_OK;
    unsigned long long total = 0;
    HIPCHK(c, hipMemcpyAsync(&total, h.d_misc + 1, 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const long long cap = h.cfg.hitlog_capacity;
    const long long have = (long long)std::min<unsigned long long>(total, (unsigned long long)cap);
    const long long take = std::min<long long>(have, max);
    std::vector<int32_t> all((size_t)cap * 6);
    HIPCHK(c, hipMemcpyAsync(all.data(), h.d_hits, all.size() * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const long long first = (long long)total - take;
    for (long long k = 0; k < take; k++) {
        const long long slot = (first + k) % cap;
        memcpy(&out[k], &all[(size_t)slot * 6], sizeof(pic_hit));
    }
    *n = take;
    return PIC_OK;
}

pic_status pic_batch_solve_info(pic_ctx *c, int32_t i, pic_solve_info *out)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (!out || i < 0 || i >= c->n) return fail(c, PIC_ERR_ARG, "bad instance or output");
    *out = c->in[i].last;
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
    if (c->d_inst) (void)hipStreamSynchronize(c->stream);
    if (c->bin_stream) (void)hipStreamSynchronize(c->bin_stream);
    for (auto &kv : c->outer_graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : c->chunk_graphs) (void)hipGraphExecDestroy(kv.second);
    for (auto &kv : c->step_graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->bin_stream) (void)hipStreamDestroy(c->bin_stream);
    if (c->ev_bin_go) (void)hipEventDestroy(c->ev_bin_go);
    if (c->ev_bin_done) (void)hipEventDestroy(c->ev_bin_done);
    for (auto e : c->ev0) if (e) (void)hipEventDestroy(e);
    for (auto e : c->ev1) if (e) (void)hipEventDestroy(e);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    delete c;
}

} // extern "C"

// Internal (C++ linkage, not exported by the headers): see ctx_view.h.
pic_status pic_ctx_view(pic_ctx *c, int i, PicCtxView *out)
{
    if (check(c) != PIC_OK) return PIC_ERR_STATE;
    if (i < 0 || i >= c->n || !out) return fail(c, PIC_ERR_ARG, "bad instance or output");
    const InstHost &h = c->in[i];
    out->phi = h.buf.phi;
    out->phi_prev = c->have_prev ? h.d_phi_prev : nullptr;
    out->b = h.buf.b;
    out->node_cond = h.d_node_cond;
    out->NX = h.g.NX;
    out->NY = h.g.NY;
    out->px = h.g.px;
    out->py = h.g.py;
    out->stream = c->stream;
    return PIC_OK;
}

