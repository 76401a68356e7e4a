// gfx950 kernels of the 2D electrostatic PIC step (arXiv:1610.03918, Sec. II).
//
// Every kernel serves a batch of independent instances: per-instance state
// is read from a device array of Inst descriptors, and a launch covers the
// blocks of several units (instances, or instance x species pairs) listed in
// a Tab.  Grid kernels work on node grids (NX x NY, row-major in x) with
// 64x4 thread blocks; floating-point reductions are float64 block partials
// summed in block order by a one-block-per-unit finalize kernel, so every
// result is reproducible bit for bit.  The particle kernel processes one tile
// of cells per block, accumulating the area-weighting moments of its
// particles in LDS as integers and flushing them to the int64 node charge
// with atomics (exact, order-free).
//
// Compiled with -ffp-contract=off: every float operation of the push is
// rounded in the order written.
#include "pic_internal.h"

namespace pic {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int wrap_lo(int a, int n) { return a < 0 ? a + n : a; }
__device__ __forceinline__ int wrap_hi(int a, int n) { return a >= n ? a - n : a; }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Unit of a launch that owns block b (uniform per block).
__device__ __forceinline__ int unit_of(const Tab &t, int b)
{
    int k = 0;
    while (k + 1 < t.n && b >= t.boff[k + 1]) k++;
    return k;
}

static inline int tab_blocks(const Tab &t) { return t.boff[t.n]; }

// Grid kernels: node (i, j) of the unit that owns this block.
#define GRID_BEGIN(t)                                                        \
    const int ku = unit_of(t, (int)blockIdx.x);                              \
    const int lb = (int)blockIdx.x - t.boff[ku];                             \
    const int byb = lb / t.bx[ku], bxb = lb - byb * t.bx[ku];                \
    const int j = bxb * kGridBX + (int)threadIdx.x;                          \
    const int i = byb * kGridBY + (int)threadIdx.y;                          \
    const Inst &I = insts[t.id[ku]];

#define NODE_IDX(NX_, NY_)                                                   \
    const int NX = (NX_), NY = (NY_);                                        \
    const bool inb = (i < NX) && (j < NY);                                   \
    const long long n = (long long)i * NY + j;

static inline dim3 gblock() { return dim3(kGridBX, kGridBY); }

// Writes this block's sums of NQ per-thread values (fixed tree order) to
// pt.p[q * stride + block].  k_finalize adds a unit's partials in block order.
template <int NQ>
__device__ void block_partials(const double (&val)[NQ], const Part &pt)
{
    __shared__ double sh[NQ][16];
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int nt = blockDim.x * blockDim.y;
    const int lane = tid & 63, wid = tid >> 6, nw = (nt + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NQ; q++) {
        double v = wave_sum(val[q]);
        if (lane == 0) sh[q][wid] = v;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            double s = 0.0;
            for (int w = 0; w < nw; w++) s += sh[q][w];
            pt.p[q * pt.stride + blockIdx.x] = s;
        }
    }
}

// Scalar logic of operation op on one instance, from the totals t0, t1 of
// its partials (one thread).
__device__ void apply_op(const Inst &I, int op, double t0, double t1)
{
    double *S = I.S;
    int *F = I.F;
    if ((op == OP_PQ || op == OP_UPDATE || op == OP_RZ) && F[F_DONE]) return;
    if (op == OP_RR64_PASS && F[F_SKIP]) return;
    if (op == OP_INIT && F[F_CONV]) {
        F[F_SKIP] = 1;
        F[F_DONE] = 1;
        return;
    }
    const double bb = S[S_BB] > 0.0 ? S[S_BB] : 1.0;
    const double tol2 = I.rtol * I.rtol;
    switch (op) {
    case OP_ASM:
        if (I.g.px && I.g.py) S[S_SUM] = t1;
        else S[S_BB] = t0;
        break;
    case OP_BB_PER: S[S_BB] = t0; break;
    case OP_SUM: S[S_SUM] = t0; break;
    case OP_RR64_START:
        // ||b||^2 of the right-hand side being solved (b may have been written
        // by the caller since the last assembly)
        S[S_BB] = t1;
        S[S_RR64] = t0;
        S[S_RELRES0] = t0;
        F[F_CONV] = (t0 <= tol2 * (t1 > 0.0 ? t1 : 1.0)) ? 1 : 0;
        F[F_ITER_TOT] = 0;
        F[F_PASSES] = 0;
        F[F_ITER1] = 0;
        F[F_DONE] = 0;
        F[F_SKIP] = 0;
        break;
    case OP_RR64_PASS:
        S[S_RR64] = t0;
        F[F_CONV] = (t0 <= tol2 * bb) ? 1 : 0;
        break;
    case OP_INIT: {
        // inner stop ratio: 0.3 rtol / relres, kept within [eta_min, 0.5]
        double eta2 = 0.09 * tol2 * bb / (S[S_RR64] > 0.0 ? S[S_RR64] : 1.0);
        const double lo = I.eta_min * I.eta_min;
        eta2 = eta2 < lo ? lo : (eta2 > 0.25 ? 0.25 : eta2);
        F[F_SKIP] = 0;
        S[S_ETA2] = eta2;
        S[S_RR0] = t0;
        S[S_RR] = t0;
        F[F_DONE] = (t0 == 0.0) ? 1 : 0;
        F[F_ITER] = 0;
        F[F_PASSES] += 1;
        if (!I.mg) { S[S_RZOLD] = S[S_RZ]; S[S_RZ] = t1; }
        break;
    }
    case OP_PQ: S[S_PQ] = t0; break;
    case OP_UPDATE:
        if (I.mg && !(S[S_CG_NALPHA] > 0.0 && S[S_CG_NALPHA] < INFINITY && S[S_CG_NBETA] < INFINITY)) {
            // the step had no usable length (the level-0 down kernel skipped it)
            F[F_DONE] = 1;
            break;
        }
        S[S_RR] = t0;
        F[F_ITER] += 1;
        F[F_ITER_TOT] += 1;
        if (F[F_PASSES] == 1) F[F_ITER1] = F[F_ITER];
        if (t0 <= S[S_ETA2] * S[S_RR0]) F[F_DONE] = 1;
        if (!I.mg) { S[S_RZOLD] = S[S_RZ]; S[S_RZ] = t1; }
        else {
            // the step's alpha, beta and r.z, computed by the level-0 down kernel
            S[S_CG_ALPHA] = S[S_CG_NALPHA];
            S[S_CG_BETA] = S[S_CG_NBETA];
            S[S_CG_GAMMA] = S[S_CG_NGAMMA];
        }
        break;
    case OP_RZ: S[S_RZOLD] = S[S_RZ]; S[S_RZ] = t0; break;
    }
}

// One block per unit: totals of the unit's partials in block order, then the
// scalar logic of the operation on that instance.
// Sums of the partials b0 .. b1-1 of nq quantities by threads 0 .. 255 of a
// block (others pass through): per-thread sums in a fixed order, then one
// per wavefront into sh[q][0 .. 3].  The caller synchronises and adds the
// four, so every kernel that reduces the same partials gets the same totals.
__device__ __forceinline__ void partial_sums_256(const Part &pt, int b0, int b1, int nq, double (*sh)[4], int tid)
{
    if (tid >= 256) return;
    const int lane = tid & 63, wid = tid >> 6;
    double s[2] = {0.0, 0.0};
    // loads of a round issued together
    for (int k0 = b0; k0 < b1; k0 += 8 * 256) {
        double v[2][8];
#pragma unroll
        for (int r = 0; r < 8; r++) {
            const int k = k0 + r * 256 + tid;
            v[0][r] = k < b1 ? pt.p[k] : 0.0;
            v[1][r] = (nq > 1 && k < b1) ? pt.p[pt.stride + k] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; r++) {
            s[0] += v[0][r];
            s[1] += v[1][r];
        }
    }
    for (int q = 0; q < 2; q++) {
        const double w = wave_sum(s[q]);
        if (lane == 0) sh[q][wid] = w;
    }
}

// Chronopoulos-Gear recurrences of the multigrid-preconditioned CG from
// gamma = r.z and delta = (A z).z of the last V-cycle: beta = gamma /
// gamma_old, alpha = gamma / (delta - beta gamma / alpha_old) (= r.z / p.Ap);
// on the first step alpha = gamma / delta, beta = 0.  False when the step
// length is not positive and finite (the inner solve ends there; the float64
// refinement carries on).
__device__ __forceinline__ bool cg_coefficients(const double *S, int iter, double gamma, double delta,
                                                double &alpha, double &beta)
{
    beta = 0.0;
    if (iter == 0) {
        alpha = gamma / delta;
    } else {
        beta = gamma / S[S_CG_GAMMA];
        alpha = gamma / (delta - beta * gamma / S[S_CG_ALPHA]);
    }
    return alpha > 0.0 && alpha < INFINITY && beta < INFINITY;
}

__global__ __launch_bounds__(256) void k_finalize(const Inst *insts, Tab t, Part pt, int op)
{
    const Inst &I = insts[t.id[blockIdx.x]];
    const int *F = I.F;
    const bool inner = op == OP_PQ || op == OP_UPDATE || op == OP_RZ;
    if (inner && F[F_DONE]) return;
    if (op == OP_RR64_PASS && F[F_SKIP]) return;
    if (op == OP_INIT && F[F_CONV]) {
        if (threadIdx.x == 0) apply_op(I, op, 0.0, 0.0);
        return;
    }
    __shared__ double sh[2][4];
    const int tid = threadIdx.x;
    const int nq = (op == OP_ASM || op == OP_INIT || op == OP_UPDATE || op == OP_RR64_START) ? 2 : 1;
    partial_sums_256(pt, t.boff[blockIdx.x], t.boff[blockIdx.x + 1], nq, sh, tid);
    __syncthreads();
    if (tid != 0) return;
    apply_op(I, op, sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3], sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]);
}

static void finalize(const Inst *I, const Tab &t, Part pt, int op, hipStream_t s)
{
    if (t.n > 0) hipLaunchKernelGGL(k_finalize, dim3(t.n), dim3(256), 0, s, I, t, pt, op);
}

__global__ void k_zero_u64(unsigned long long *p, long long n)
{
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long st = (long long)gridDim.x * blockDim.x;
    for (; k < n; k += st) p[k] = 0ull;
}

void launch_zero_u64(unsigned long long *p, long long n, hipStream_t s)
{
    if (n <= 0) return;
    long long nb = (n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)nb), dim3(256), 0, s, p, n);
}

__global__ void k_tick(long long *step) { *step += 1; }

void launch_tick(long long *step, hipStream_t s)
{
    hipLaunchKernelGGL(k_tick, dim3(1), dim3(1), 0, s, step);
}

// ---------------------------------------------------------------------------
// field: E = -grad(phi) at the four corners of every cell (Sec. II)
// ---------------------------------------------------------------------------

// One axis of -grad(phi) at a node.  Inside: central difference.  At a
// Dirichlet node: two-point difference toward the only free neighbour if
// exactly one neighbour is free; central if both neighbours exist (zero along
// an equipotential wall); two-point with the only neighbour at a domain edge.
__device__ __forceinline__ double axis_field(double pm, double pc, double pp, bool hm, bool hp,
                                             bool fm, bool fp, bool fixed)
{
    if (!fixed) return -(pp - pm) * 0.5;
    if (hm && hp) {
        if (fp && !fm) return -(pp - pc);
        if (fm && !fp) return -(pc - pm);
        return -(pp - pm) * 0.5;
    }
    if (hp) return -(pp - pc);
    if (hm) return -(pc - pm);
    return 0.0;
}

__device__ __forceinline__ float2 node_field(const Geom g, const uint8_t *nc, const double *phi,
                                             int i, int j)
{
    const int NX = g.NX, NY = g.NY;
    const long long n = (long long)i * NY + j;
    const bool fixed = nc[n] != 0;
    const double pc = phi[n];
    bool hm = g.px || i > 0, hp = g.px || i < NX - 1;
    int im = g.px ? wrap_lo(i - 1, NX) : i - 1, ip = g.px ? wrap_hi(i + 1, NX) : i + 1;
    double pm = hm ? phi[(long long)im * NY + j] : 0.0;
    double pp = hp ? phi[(long long)ip * NY + j] : 0.0;
    bool fm = hm && nc[(long long)im * NY + j] == 0;
    bool fp = hp && nc[(long long)ip * NY + j] == 0;
    double ex = axis_field(pm, pc, pp, hm, hp, fm, fp, fixed);
    bool gm = g.py || j > 0, gp = g.py || j < NY - 1;
    int jm = g.py ? wrap_lo(j - 1, NY) : j - 1, jp = g.py ? wrap_hi(j + 1, NY) : j + 1;
    double qm = gm ? phi[(long long)i * NY + jm] : 0.0;
    double qp = gp ? phi[(long long)i * NY + jp] : 0.0;
    bool em = gm && nc[(long long)i * NY + jm] == 0;
    bool ep = gp && nc[(long long)i * NY + jp] == 0;
    double ey = axis_field(qm, pc, qp, gm, gp, em, ep, fixed);
    return make_float2((float)ex, (float)ey);
}

// One thread per cell; writes the cell's four corner fields (float32, each
// node's computed once per block) and,
// when requested (the field of a push), clears both species' node charge for
// the coming deposit.  The field of a push also counts, in F_UNCONV, a
// potential whose last residual test failed, and keeps the largest such
// relative residual in S_WORST (one thread per instance).
__global__ void k_field(const Inst *insts, Tab t, int zero_rho)
{
    GRID_BEGIN(t)
    const Geom g = I.g;
    if (zero_rho && i == 0 && j == 0 && !I.F[F_CONV]) {
        I.F[F_UNCONV] += 1;
        const double bb = I.S[S_BB] > 0.0 ? I.S[S_BB] : 1.0;
        const double rel = sqrt(I.S[S_RR64] / bb);
        if (!(rel <= I.S[S_WORST])) I.S[S_WORST] = rel;
    }
    if (zero_rho && i < g.NX && j < g.NY) {
        const long long n = (long long)i * g.NY + j;
        I.rho[0][n] = 0ull;
        I.rho[1][n] = 0ull;
    }
    // the field of each node of the block's (kGridBY + 1) x (kGridBX + 1)
    // corner set, once, in LDS; a periodic axis wraps the far row / column
    const uint8_t *nc = I.node_cond;
    const double *phi = I.phi;
    __shared__ float2 sn[kGridBY + 1][kGridBX + 1];
    const int ti = (int)threadIdx.y, tj = (int)threadIdx.x;
    auto node_at = [&](int a, int b) {
        if (g.px && a >= g.NX) a %= g.NX;
        if (g.py && b >= g.NY) b %= g.NY;
        return (a < g.NX && b < g.NY) ? node_field(g, nc, phi, a, b) : make_float2(0.f, 0.f);
    };
    sn[ti][tj] = node_at(i, j);
    if (ti == 0) sn[kGridBY][tj] = node_at(i - ti + kGridBY, j);
    if (ti == 1 && tj <= kGridBY) sn[tj][kGridBX] = node_at(i - ti + tj, j - tj + kGridBX);
    __syncthreads();
    if (i >= g.nx || j >= g.ny) return;
    const float2 e00 = sn[ti][tj], e10 = sn[ti + 1][tj], e01 = sn[ti][tj + 1], e11 = sn[ti + 1][tj + 1];
    const long long c = (long long)i * g.ny + j;
    I.E4[2 * c] = make_float4(e00.x, e00.y, e10.x, e10.y);
    I.E4[2 * c + 1] = make_float4(e01.x, e01.y, e11.x, e11.y);
}

void launch_field(const Inst *I, const Tab &t, int zero_rho, hipStream_t s)
{
    if (t.n) hipLaunchKernelGGL(k_field, dim3(tab_blocks(t)), gblock(), 0, s, I, t, zero_rho);
}

// ---------------------------------------------------------------------------
// assemble: b = (N_i - N_e) w 2^-32 + Dirichlet lifts (eq. 5, unit spacing)
// V: conductor potentials, 8 per instance (indexed by instance id)
// ---------------------------------------------------------------------------

// V: conductor potentials of every step of the table window, indexed
// ((step - base) * ninst + instance) * 8 with the device step counter.
// A window row outside [0, vwin) (the runtime never launches one) sets the
// instance's kErrVWindow error bit, which the host reports as PIC_ERR_STATE
// at its next look at the flags; the read itself stays inside the table.
__global__ void k_assemble(const Inst *insts, Tab t, const double *Vtab, const long long *ctl,
                           int ninst, int vwin, Part pt)
{
    GRID_BEGIN(t)
    const Geom g = I.g;
    NODE_IDX(g.NX, g.NY)
    long long row = ctl[0] - ctl[1];
    if (row < 0 || row >= vwin) {
        if (i == 0 && j == 0) I.F[F_ERR] |= kErrVWindow;
        row = 0;
    }
    const double *V = Vtab + (row * ninst + t.id[ku]) * 8;
    double bb = 0.0, sm = 0.0;
    if (inb) {
        const uint8_t *nc = I.node_cond;
        const int c = nc[n];
        if (c) {
            I.b[n] = V[c];
            I.phi[n] = V[c];
        } else {
            long long Ni = (long long)I.rho[1][n];
            if (I.charge_mode == 2 && i == I.charge_row) {
                const int jl = g.py ? wrap_lo(j - 1, g.ny) : j - 1;
                if (j < g.ny) Ni += (long long)I.surf[j] << 31;
                if (jl >= 0) Ni += (long long)I.surf[jl] << 31;
            }
            double r = (double)(Ni - (long long)I.rho[0][n]) * I.qcharge;
            if (I.charge_mode == 1 && i == I.charge_row && j >= I.sjl && j <= I.sjh) r += I.sden;
            const int im = g.px ? wrap_lo(i - 1, NX) : i - 1, ip = g.px ? wrap_hi(i + 1, NX) : i + 1;
            const int jm = g.py ? wrap_lo(j - 1, NY) : j - 1, jp = g.py ? wrap_hi(j + 1, NY) : j + 1;
            int cn;
            if ((cn = nc[(long long)im * NY + j])) r += V[cn];
            if ((cn = nc[(long long)ip * NY + j])) r += V[cn];
            if ((cn = nc[(long long)i * NY + jm])) r += V[cn];
            if ((cn = nc[(long long)i * NY + jp])) r += V[cn];
            I.b[n] = r;
            if (!I.lev[0].fix[n]) bb = r * r;
            sm = r;
        }
    }
    double v[2] = {bb, sm};
    block_partials<2>(v, pt);
}

void launch_assemble(const Inst *I, const Tab &t, const double *Vtab, const long long *ctl,
                     int ninst, int vwin, Part pt, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_assemble, dim3(tab_blocks(t)), gblock(), 0, s, I, t, Vtab, ctl, ninst, vwin,
                       pt);
    finalize(I, t, pt, OP_ASM, s);
}

// Fully periodic grid: the source must have zero mean (gauge); subtract it
// and form ||b||^2 over the unknowns (the pinned node excluded).
__global__ void k_project_mean(const Inst *insts, Tab t, Part pt)
{
    GRID_BEGIN(t)
    NODE_IDX(I.g.NX, I.g.NY)
    const double mean = I.S[S_SUM] / ((double)NX * (double)NY);
    double bb = 0.0;
    if (inb) {
        const double r = I.b[n] - mean;
        I.b[n] = r;
        if (!I.lev[0].fix[n]) bb = r * r;
    }
    double v[1] = {bb};
    block_partials<1>(v, pt);
}

void launch_project_mean(const Inst *I, const Tab &t, Part pt, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_project_mean, dim3(tab_blocks(t)), gblock(), 0, s, I, t, pt);
    finalize(I, t, pt, OP_BB_PER, s);
}

__global__ void k_sum_phi(const Inst *insts, Tab t, Part pt)
{
    GRID_BEGIN(t)
    NODE_IDX(I.g.NX, I.g.NY)
    double v[1] = {inb ? I.phi[n] : 0.0};
    block_partials<1>(v, pt);
}

// phi -= S[slot] * (mean ? 1 / (NX NY) : 1) on every node
__global__ void k_shift_phi(const Inst *insts, Tab t, int slot, int mean)
{
    GRID_BEGIN(t)
    NODE_IDX(I.g.NX, I.g.NY)
    const double sc = mean ? 1.0 / ((double)NX * (double)NY) : 1.0;
    if (inb) I.phi[n] -= I.S[slot] * sc;
}

__global__ void k_read_node0(const Inst *insts, Tab t)
{
    const Inst &I = insts[t.id[blockIdx.x]];
    I.S[S_PIN] = I.phi[0];
}

void launch_shift_mean(const Inst *I, const Tab &t, Part pt, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_sum_phi, dim3(tab_blocks(t)), gblock(), 0, s, I, t, pt);
    finalize(I, t, pt, OP_SUM, s);
    hipLaunchKernelGGL(k_shift_phi, dim3(tab_blocks(t)), gblock(), 0, s, I, t, (int)S_SUM, 1);
}

// Fully periodic grid: node 0 is held at 0 during the solve (gauge); shift a
// start so that it already satisfies that.
void launch_pin_shift(const Inst *I, const Tab &t, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_read_node0, dim3(t.n), dim3(1), 0, s, I, t);
    hipLaunchKernelGGL(k_shift_phi, dim3(tab_blocks(t)), gblock(), 0, s, I, t, (int)S_PIN, 0);
}

// Start of the solve on the unknowns; on a fully periodic grid also on the
// pinned node (the gauge shift that follows moves it back to 0).  kind 0:
// zero; kind 2: copy from guess (single-unit launches only).
__global__ void k_set_guess(const Inst *insts, Tab t, int kind, const double *guess)
{
    GRID_BEGIN(t)
    NODE_IDX(I.g.NX, I.g.NY)
    if (!inb || (I.lev[0].fix[n] && !(I.g.px && I.g.py))) return;
    I.phi[n] = (kind == 0) ? 0.0 : guess[n];
}

void launch_set_guess(const Inst *I, const Tab &t, int kind, const double *guess, hipStream_t s)
{
    if (t.n) hipLaunchKernelGGL(k_set_guess, dim3(tab_blocks(t)), gblock(), 0, s, I, t, kind, guess);
}

// Linear extrapolation in time of the unknowns: phi <- 2 phi - prev and
// prev <- phi (the previous step's solution); with have_prev = 0 only the
// copy is made.
__global__ void k_extrapolate(const Inst *insts, Tab t, int have_prev)
{
    GRID_BEGIN(t)
    NODE_IDX(I.g.NX, I.g.NY)
    if (!inb || (I.lev[0].fix[n] && !(I.g.px && I.g.py))) return;
    const double v = I.phi[n];
    if (have_prev) I.phi[n] = 2.0 * v - I.phi_prev[n];
    I.phi_prev[n] = v;
}

void launch_extrapolate(const Inst *I, const Tab &t, int have_prev, hipStream_t s)
{
    if (t.n) hipLaunchKernelGGL(k_extrapolate, dim3(tab_blocks(t)), gblock(), 0, s, I, t, have_prev);
}

// ---------------------------------------------------------------------------
// float64 outer residual: r = b - A phi on the unknowns, ||r||^2 (float64),
// r rounded to float32 for the inner preconditioned CG; at the start of a
// solve also ||b||^2 over the unknowns (the reference of the tolerance).
// A = 4 - (sum of free neighbours); fixed neighbours sit in b already.
// ---------------------------------------------------------------------------

__global__ void k_resid64(const Inst *insts, Tab t, int after_pass, Part pt)
{
    GRID_BEGIN(t)
    if (after_pass && I.F[F_SKIP]) return;
    NODE_IDX(I.g.NX, I.g.NY)
    const uint8_t *fix = I.lev[0].fix;
    const double *phi = I.phi;
    double rr = 0.0, bsq = 0.0;
    if (inb) {
        if (fix[n]) {
            I.lev[0].g[n] = 0.0f;
        } else {
            bsq = I.b[n] * I.b[n];
            const int im = wrap_lo(i - 1, NX), ip = wrap_hi(i + 1, NX);
            const int jm = wrap_lo(j - 1, NY), jp = wrap_hi(j + 1, NY);
            const long long a = (long long)im * NY + j, c = (long long)ip * NY + j;
            const long long d = (long long)i * NY + jm, e = (long long)i * NY + jp;
            double s = 4.0 * phi[n];
            if (!fix[a]) s -= phi[a];
            if (!fix[c]) s -= phi[c];
            if (!fix[d]) s -= phi[d];
            if (!fix[e]) s -= phi[e];
            const double r = I.b[n] - s;
            I.lev[0].g[n] = (float)r;
            rr = r * r;
        }
    }
    double v[2] = {rr, bsq};
    block_partials<2>(v, pt);
}

void launch_resid64(const Inst *I, const Tab &t, int after_pass, Part pt, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_resid64, dim3(tab_blocks(t)), gblock(), 0, s, I, t, after_pass, pt);
    finalize(I, t, pt, after_pass ? OP_RR64_PASS : OP_RR64_START, s);
}

// ---------------------------------------------------------------------------
// the paper's own iterations for eq. (5) (Sec. II): Jacobi and Gauss-Seidel
// sweeps of the masked 5-point system in float64.  A free node takes
// (b + sum of its free neighbours) / 4 with the neighbours added in the order
// x-1, x+1, y-1, y+1 (fixed neighbours' potentials sit in b); Gauss-Seidel
// visits the red nodes (i + j even), then the black ones.  An instance whose
// float64 residual already met rtol is left alone.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double sweep_value(const double *src, const double *b, const uint8_t *fix, int i,
                                              int j, int NX, int NY, long long n)
{
    const int im = wrap_lo(i - 1, NX), ip = wrap_hi(i + 1, NX);
    const int jm = wrap_lo(j - 1, NY), jp = wrap_hi(j + 1, NY);
    const long long a = (long long)im * NY + j, c = (long long)ip * NY + j;
    const long long d = (long long)i * NY + jm, e = (long long)i * NY + jp;
    double s = b[n];
    if (!fix[a]) s += src[a];
    if (!fix[c]) s += src[c];
    if (!fix[d]) s += src[d];
    if (!fix[e]) s += src[e];
    return s * 0.25;
}

// One Jacobi sweep: dir 0 reads phi and writes phi2, dir 1 the reverse.
__global__ void k_jacobi64(const Inst *insts, Tab t, int dir)
{
    GRID_BEGIN(t)
    if (I.F[F_CONV]) return;
    NODE_IDX(I.g.NX, I.g.NY)
    if (!inb) return;
    const double *src = dir ? I.phi2 : I.phi;
    double *dst = dir ? I.phi : I.phi2;
    const uint8_t *fix = I.lev[0].fix;
    dst[n] = fix[n] ? src[n] : sweep_value(src, I.b, fix, i, j, NX, NY, n);
}

// One colour of a red-black Gauss-Seidel sweep, in place.
__global__ void k_gs64(const Inst *insts, Tab t, int col)
{
    GRID_BEGIN(t)
    if (I.F[F_CONV]) return;
    NODE_IDX(I.g.NX, I.g.NY)
    if (!inb || ((i + j) & 1) != col) return;
    const uint8_t *fix = I.lev[0].fix;
    if (!fix[n]) I.phi[n] = sweep_value(I.phi, I.b, fix, i, j, NX, NY, n);
}

void launch_sweeps(const Inst *I, const Tab &t, int jacobi, int sweeps, hipStream_t s)
{
    if (!t.n) return;
    for (int k = 0; k < sweeps; k++) {
        if (jacobi) {
            hipLaunchKernelGGL(k_jacobi64, dim3(tab_blocks(t)), gblock(), 0, s, I, t, k & 1);
        } else {
            hipLaunchKernelGGL(k_gs64, dim3(tab_blocks(t)), gblock(), 0, s, I, t, 0);
            hipLaunchKernelGGL(k_gs64, dim3(tab_blocks(t)), gblock(), 0, s, I, t, 1);
        }
    }
}

__global__ void k_phi_update(const Inst *insts, Tab t)
{
    GRID_BEGIN(t)
    if (I.F[F_SKIP]) return;
    NODE_IDX(I.g.NX, I.g.NY)
    if (inb && !I.lev[0].fix[n]) I.phi[n] += (double)I.e[n];
}

void launch_phi_update(const Inst *I, const Tab &t, hipStream_t s)
{
    if (t.n) hipLaunchKernelGGL(k_phi_update, dim3(tab_blocks(t)), gblock(), 0, s, I, t);
}

// ---------------------------------------------------------------------------
// multigrid pieces on any level (generic pointers: global or LDS)
//   stencil per level: 4u - sum(free neighbours) = g   (h^2 folded into g)
//   restriction g_c = P^T r (weights 1, 1/2, 1/4), prolongation bilinear P,
//   red-black Gauss-Seidel: pre red->black, post black->red (symmetric)
// ---------------------------------------------------------------------------

struct Nb {
    int im, ip, jm, jp;
};

__device__ __forceinline__ Nb nbs(int i, int j, int NX, int NY)
{
    Nb r;
    r.im = wrap_lo(i - 1, NX);
    r.ip = wrap_hi(i + 1, NX);
    r.jm = wrap_lo(j - 1, NY);
    r.jp = wrap_hi(j + 1, NY);
    return r;
}

// Bilinear prolongation of the coarse correction e at a red fine node
// (both indices even: coincident node; both odd: cell centre).
__device__ __forceinline__ float prolong_red(const float *e, int NXc, int NYc, int a, int c)
{
    int I = a >> 1, J = c >> 1;
    if (((a | c) & 1) == 0) return e[(long long)I * NYc + J];
    int I1 = wrap_hi(I + 1, NXc), J1 = wrap_hi(J + 1, NYc);
    return 0.25f * (e[(long long)I * NYc + J] + e[(long long)I1 * NYc + J] +
                    e[(long long)I * NYc + J1] + e[(long long)I1 * NYc + J1]);
}

// ---------------------------------------------------------------------------
// preconditioned CG on level 0 (float32 vectors, float64 dot products)
// ---------------------------------------------------------------------------

// Inner start: e = 0, z = red-from-zero of M r (or z = r/4 without MG),
// ||r||^2 and r.z partials.  Skipped once the float64 residual converged.
__global__ void k_init_red0(const Inst *insts, Tab t, Part pt)
{
    GRID_BEGIN(t)
    if (I.F[F_CONV]) return;
    const LevelDev L = I.lev[0];
    NODE_IDX(L.NX, L.NY)
    const int mg = I.mg;
    double rr = 0.0, rz = 0.0;
    if (inb) {
        const float r = L.g[n];
        I.e[n] = 0.0f;
        float z = 0.0f;
        if (!L.fix[n]) {
            rr = (double)r * (double)r;
            if (!mg || (((i + j) & 1) == 0)) z = r * 0.25f;
            rz = (double)r * (double)z;
        }
        L.u[n] = z;
    }
    double v[2] = {rr, rz};
    block_partials<2>(v, pt);
}

void launch_init_red0(const Inst *I, const Tab &t, Part pt, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_init_red0, dim3(tab_blocks(t)), gblock(), 0, s, I, t, pt);
    finalize(I, t, pt, OP_INIT, s);
}

// p_new = z + beta p_old, q = A p_new, p.q  (beta = rz / rz_old; 0 on the first)
__global__ void k_pupdate_Ap(const Inst *insts, Tab t, int kold, int first, Part pt)
{
    GRID_BEGIN(t)
    if (I.F[F_DONE]) return;
    const LevelDev L = I.lev[0];
    NODE_IDX(L.NX, L.NY)
    const float *p_old = I.p[kold];
    float *p_new = I.p[1 - kold];
    float *q = I.q;
    const float beta = first ? 0.0f : (float)(I.S[S_RZ] / I.S[S_RZOLD]);
    double pq = 0.0;
    if (inb) {
        if (L.fix[n]) {
            p_new[n] = 0.0f;
            q[n] = 0.0f;
        } else {
            Nb b = nbs(i, j, NX, NY);
            const long long m[4] = {(long long)b.im * NY + j, (long long)b.ip * NY + j,
                                    (long long)i * NY + b.jm, (long long)i * NY + b.jp};
            const float *z = I.z;
            const float pc = first ? z[n] : z[n] + beta * p_old[n];
            float s = 4.0f * pc;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                if (L.fix[m[k]]) continue;
                const float pn = first ? z[m[k]] : z[m[k]] + beta * p_old[m[k]];
                s -= pn;
            }
            p_new[n] = pc;
            q[n] = s;
            pq = (double)pc * (double)s;
        }
    }
    double v[1] = {pq};
    block_partials<1>(v, pt);
}

void launch_pupdate_Ap(const Inst *I, const Tab &t, int kold, int first, Part pt, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_pupdate_Ap, dim3(tab_blocks(t)), gblock(), 0, s, I, t, kold, first, pt);
    finalize(I, t, pt, OP_PQ, s);
}

// alpha = rz / pq; e += alpha p; r -= alpha q; ||r||^2; z = red-from-zero of
// M r (or r/4 without MG, with r.z).  The finalize marks the inner solve
// done when ||r||^2 <= eta^2 ||r0||^2 and counts the iteration.
__global__ void k_update_red0(const Inst *insts, Tab t, int knew, Part pt)
{
    GRID_BEGIN(t)
    if (I.F[F_DONE]) return;
    const LevelDev L = I.lev[0];
    NODE_IDX(L.NX, L.NY)
    const int mg = I.mg;
    const float *p = I.p[knew];
    const float alpha = (float)(I.S[S_RZ] / I.S[S_PQ]);
    double rr = 0.0, rz = 0.0;
    if (inb) {
        float z = 0.0f;
        if (!L.fix[n]) {
            I.e[n] = I.e[n] + alpha * p[n];
            const float r = L.g[n] - alpha * I.q[n];
            L.g[n] = r;
            rr = (double)r * (double)r;
            if (!mg || (((i + j) & 1) == 0)) z = r * 0.25f;
            rz = (double)r * (double)z;
        }
        L.u[n] = z;
    }
    double v[2] = {rr, rz};
    block_partials<2>(v, pt);
}

void launch_update_red0(const Inst *I, const Tab &t, int knew, Part pt, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_update_red0, dim3(tab_blocks(t)), gblock(), 0, s, I, t, knew, pt);
    finalize(I, t, pt, OP_UPDATE, s);
}

// ---------------------------------------------------------------------------
// fused V-cycle kernels for the fine levels, one block per 32 x 32 tile of the
// fine level (launch table: tiles, bx = tiles across y).  Each block stages a
// window of u, g and the mask around its tile in LDS (periodic axes wrap, nodes
// outside a bounded axis enter as fixed), recomputes in the window what it
// needs, and writes only its own tile (or its own coarse nodes).  Each
// launch reads one buffer of the level and writes the other, so no block sees
// another block's writes:
//   down: u (red-from-zero start) -> pre-smoothing (black, then red + black
//         NU - 1 times) -> uo, and the restricted residual to level l + 1
//   up:   uo -> black update with the prolonged coarse correction, then red,
//         then black + red NU - 1 times -> u (on level 0 the CG's z, with
//         the r.z partials)
// The post-smoothing is the pre-smoothing's colour sequence reversed, which
// keeps the V-cycle symmetric.
// Arithmetic per node: Gauss-Seidel value (g + neighbours) / 4 with the
// neighbours added in the order x-1, x+1, y-1, y+1; restriction = sum over
// the red fine nodes of the 3 x 3 stencil of weight x residual (centre 1,
// diagonals 1/4; the black residuals vanish after a black half-sweep);
// bilinear prolongation of the coarse correction onto the red nodes.
// ---------------------------------------------------------------------------

constexpr int kMgTile = 32;
constexpr int kMgThreads = 512;

__device__ __forceinline__ int wrap_any(int x, int n) { return ((x % n) + n) % n; }

// Window index (wi0 + a, wj0 + c) -> global node of level (NX, NY), or -1
// outside a bounded axis.
__device__ __forceinline__ long long win_node(int NX, int NY, int px, int py, int gi, int gj)
{
    if (px) gi = wrap_any(gi, NX);
    else if (gi < 0 || gi >= NX) return -1;
    if (py) gj = wrap_any(gj, NY);
    else if (gj < 0 || gj >= NY) return -1;
    return (long long)gi * NY + gj;
}

// Stages u (from src), g, fix of the W x W window with origin (wi0, wj0) on
// level L.  Fixed nodes hold u = 0 on every level (no update ever writes
// them), so the stencils below add neighbours without testing their mask;
// all loads of a thread are issued before the LDS stores.
template <int W, int NT = kMgThreads>
__device__ __forceinline__ void mg_stage(const LevelDev &L, const float *src, const float *gsrc, int px, int py,
                                         int wi0, int wj0, float *su, float *sg, uint8_t *sf)
{
    constexpr int R = (W * W + NT - 1) / NT;
    float uv[R], gv[R];
    uint8_t fv[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int k = (int)threadIdx.x + r * NT;
        const int a = k / W, c = k - a * W;
        const long long n = k < W * W ? win_node(L.NX, L.NY, px, py, wi0 + a, wj0 + c) : -1;
        uv[r] = 0.0f;
        gv[r] = 0.0f;
        fv[r] = 1;
        if (n >= 0) {
            fv[r] = L.fix[n];
            uv[r] = src[n];
            gv[r] = gsrc[n];
        }
    }
#pragma unroll
    for (int r = 0; r < R; r++) {
        const int k = (int)threadIdx.x + r * NT;
        if (k < W * W) {
            su[k] = uv[r];
            sg[k] = gv[r];
            sf[k] = fv[r];
        }
    }
}

// Level 0 of the inner CG (Chronopoulos-Gear form): stages the residual
// after this iteration's update, r - alpha (w + beta s), as g and its
// red-from-zero start as u.  With `update` false the residual is r itself
// (start of a pass).  Every block evaluates the same float32 expression for
// a node, so window copies agree with the owner's stored values.
template <int W>
__device__ __forceinline__ void mg_stage_l0(const Inst &I, int update, int first, float alpha, float beta,
                                            const float *r, const float *sv, const float *wv, int wi0, int wj0,
                                            float *su, float *sg, uint8_t *sf)
{
    constexpr int R = (W * W + kMgThreads - 1) / kMgThreads;
    const LevelDev &L = I.lev[0];
    float rv[R], s_[R], w_[R];
    uint8_t fv[R];
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int k = (int)threadIdx.x + q * kMgThreads;
        const int a = k / W, c = k - a * W;
        const long long n = k < W * W ? win_node(L.NX, L.NY, I.g.px, I.g.py, wi0 + a, wj0 + c) : -1;
        rv[q] = 0.0f;
        s_[q] = 0.0f;
        w_[q] = 0.0f;
        fv[q] = 1;
        if (n >= 0) {
            fv[q] = L.fix[n];
            rv[q] = r[n];
            if (update) {
                w_[q] = wv[n];
                if (!first) s_[q] = sv[n];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; q++) {
        const int k = (int)threadIdx.x + q * kMgThreads;
        if (k >= W * W) continue;
        const int a = k / W, c = k - a * W;
        float rn = 0.0f;
        if (!fv[q]) {
            rn = rv[q];
            if (update) {
                const float sn = first ? w_[q] : w_[q] + beta * s_[q];
                rn = rn - alpha * sn;
            }
        }
        sg[k] = rn;
        su[k] = (((a + c) & 1) == 0) ? rn * 0.25f : 0.0f;
        sf[k] = fv[q];
    }
}

// Gauss-Seidel value at window node k (neighbours in the window; fixed
// neighbours contribute their zero).
template <int W>
__device__ __forceinline__ float win_gs(const float *su, const float *sg, int k)
{
    float s = sg[k];
    s += su[k - W];
    s += su[k + W];
    s += su[k - 1];
    s += su[k + 1];
    return s * 0.25f;
}

// One colour of Gauss-Seidel over window rows/cols m .. W-1-m.  The window
// origin is an even offset from an even tile corner, so (a + c) & 1 is the
// colour of the global node.
template <int W, int NT = kMgThreads>
__device__ __forceinline__ void win_sweep(float *su, const float *sg, const uint8_t *sf, int m, int col)
{
    for (int k = threadIdx.x; k < W * W; k += NT) {
        const int a = k / W, c = k - a * W;
        if (a < m || a > W - 1 - m || c < m || c > W - 1 - m || sf[k]) continue;
        if (((a + c) & 1) != col) continue;
        su[k] = win_gs<W>(su, sg, k);
    }
}

// Down half-cycle of level l with NU pre-smoothing steps: from the
// red-from-zero start, black, then (red, black) x (NU - 1); the pre-smoothed
// level goes to uo, the restricted residual to level l + 1 (g, and u = its
// red-from-zero start).
// MODE 0: level l >= 1 (start staged from u).
// MODE 1: level 0 at the start of an inner pass: r = R[0], e = 0, ||r||^2
//         (inner stop ratio and counters in the last block).
// MODE 2: level 0 after a CG step: alpha and beta from the last V-cycle's
//         dot products (partials pq), s' = w + beta s, r' = r - alpha s',
//         p = z + beta p, e += alpha p (beta = 0 on the first step), r' and
//         s' to the other buffers of the pair, ||r'||^2 partials (pt) for
//         the inner stop test.  par: buffer of the pair holding r and s.
template <int NU, int MODE>
__global__ __launch_bounds__(kMgThreads) void k_mg_down(const Inst *insts, Tab t, int level, int par, Part pt,
                                                        Part pq)
{
    constexpr int HD = 2 * NU + 1, W = kMgTile + 2 * HD - 1;
    const int ku = unit_of(t, (int)blockIdx.x);
    const Inst &I = insts[t.id[ku]];
    int *F = I.F;
    double *S = I.S;
    const int lb = (int)blockIdx.x - t.boff[ku];
    const int ti = lb / t.bx[ku], tj = lb - ti * t.bx[ku];
    const LevelDev F0 = I.lev[level], Cc = I.lev[level + 1];
    const int i0 = ti * kMgTile, j0 = tj * kMgTile;
    __shared__ float su[W * W], sg[W * W], sr[W * W];
    __shared__ uint8_t sf[W * W];
    double rr = 0.0;
    bool work = true;
    if (MODE == 1) {
        work = !F[F_CONV];
    } else {
        if (F[F_DONE]) return;
    }
    float alpha = 0.0f, beta = 0.0f;
    if (MODE == 2) {
        // this step's alpha and beta from the last V-cycle's r.z and (A z).z
        // partials (pq): every block adds them in the same order, so all
        // blocks agree.  Block 0 records them for the step's update, which
        // also ends the inner solve when they are not usable (no block of
        // this launch writes a flag the others read).
        __shared__ double shq[2][4];
        partial_sums_256(pq, t.boff[ku], t.boff[ku + 1], 2, shq, (int)threadIdx.x);
        __syncthreads();
        const double gamma = shq[0][0] + shq[0][1] + shq[0][2] + shq[0][3];
        const double delta = shq[1][0] + shq[1][1] + shq[1][2] + shq[1][3];
        double a, b;
        const bool ok = cg_coefficients(S, F[F_ITER], gamma, delta, a, b);
        if (lb == 0 && threadIdx.x == 0) {
            S[S_CG_NALPHA] = a;
            S[S_CG_NBETA] = b;
            S[S_CG_NGAMMA] = gamma;
        }
        if (!ok) return;
        alpha = (float)a;
        beta = (float)b;
    }
    if (work) {
        if (MODE == 0) {
            mg_stage<W>(F0, F0.u, F0.g, I.g.px, I.g.py, i0 - HD, j0 - HD, su, sg, sf);
        } else {
            const int first = MODE == 2 ? F[F_ITER] == 0 : 1;
            const float *r = par ? I.cg_r1 : F0.g;
            mg_stage_l0<W>(I, MODE == 2, first, alpha, beta, r, I.cg_s[par], I.cg_w, i0 - HD, j0 - HD, su, sg, sf);
            __syncthreads();
            // own tile: the vector updates and ||r'||^2 (reads the window only)
            float *rn_out = par ? F0.g : I.cg_r1;
            float *sn_out = I.cg_s[1 - par];
            for (int k = threadIdx.x; k < kMgTile * kMgTile; k += kMgThreads) {
                const int a = k / kMgTile, c = k - a * kMgTile;
                const int gi = i0 + a, gj = j0 + c;
                if (gi >= F0.NX || gj >= F0.NY) continue;
                const long long n = (long long)gi * F0.NY + gj;
                const int w = (a + HD) * W + (c + HD);
                if (MODE == 1) {
                    I.e[n] = 0.0f;
                } else if (!sf[w]) {
                    const float z = I.z[n];
                    const float pn = first ? z : z + beta * I.p[0][n];
                    const float sn = first ? I.cg_w[n] : I.cg_w[n] + beta * I.cg_s[par][n];
                    I.p[0][n] = pn;
                    I.e[n] = I.e[n] + alpha * pn;
                    sn_out[n] = sn;
                    rn_out[n] = sg[w];
                } else {
                    I.p[0][n] = 0.0f;
                    sn_out[n] = 0.0f;
                    rn_out[n] = 0.0f;
                }
                if (!sf[w]) rr += (double)sg[w] * (double)sg[w];
            }
        }
        if (MODE == 0) __syncthreads();
#pragma unroll
        for (int m = 1; m < 2 * NU; m++) {
            win_sweep<W>(su, sg, sf, m, m & 1);           // odd m: black, even m: red
            __syncthreads();
        }
        // own nodes (both colours) to uo; residuals at the red nodes the
        // restriction reads (window rows/cols 2NU .. W-1-2NU)
        for (int k = threadIdx.x; k < kMgTile * kMgTile; k += kMgThreads) {
            const int a = k / kMgTile, c = k - a * kMgTile;
            const int gi = i0 + a, gj = j0 + c;
            if (gi >= F0.NX || gj >= F0.NY) continue;
            F0.uo[(long long)gi * F0.NY + gj] = su[(a + HD) * W + (c + HD)];
        }
        for (int k = threadIdx.x; k < W * W; k += kMgThreads) {
            const int a = k / W, c = k - a * W;
            if (a < 2 * NU || a > W - 1 - 2 * NU || c < 2 * NU || c > W - 1 - 2 * NU) continue;
            if (((a + c) & 1) != 0) continue;
            float r = 0.0f;
            if (!sf[k]) {
                float q = 4.0f * su[k];
                q -= su[k - W];
                q -= su[k + W];
                q -= su[k - 1];
                q -= su[k + 1];
                r = sg[k] - q;
            }
            sr[k] = r;
        }
        __syncthreads();
        // restriction: coarse nodes (i0/2 .. i0/2+15, j0/2 .. j0/2+15)
        if (threadIdx.x < 256) {
            const int ci = threadIdx.x >> 4, cj = threadIdx.x & 15;
            const int CI = (i0 >> 1) + ci, CJ = (j0 >> 1) + cj;
            if (CI < Cc.NX && CJ < Cc.NY) {
                const long long n = (long long)CI * Cc.NY + CJ;
                float gv = 0.0f, uv = 0.0f;
                if (!Cc.fix[n]) {
                    const int k = (2 * ci + HD) * W + (2 * cj + HD);
                    float acc = 0.0f;
                    acc += 0.25f * sr[k - W - 1];
                    acc += 0.25f * sr[k - W + 1];
                    acc += 1.0f * sr[k];
                    acc += 0.25f * sr[k + W - 1];
                    acc += 0.25f * sr[k + W + 1];
                    gv = acc;
                    if (((CI + CJ) & 1) == 0) uv = gv * 0.25f;
                }
                Cc.g[n] = gv;
                Cc.u[n] = uv;
            }
        }
    }
    if (MODE == 0) return;
    double v[1] = {rr};
    block_partials<1>(v, pt);
}

// Up half-cycle of level l with NU post-smoothing steps: black from the
// corrected reds (pre-smoothed value + bilinear prolongation of level l+1's
// result u), then red, then (black, red) x (NU - 1); result to u.
// L0: level 0 of the inner CG: z = the V-cycle result on the tile and a
// one-node ring around it, z to u (the CG's z), w = A z to cg_w, r.z and w.z
// partials, the step scalars alpha and beta in the last block.  par: buffer
// of the pair holding the current residual.
template <int NU, int L0>
__global__ __launch_bounds__(kMgThreads) void k_mg_up(const Inst *insts, Tab t, int level, int par, Part pt)
{
    constexpr int HU = 2 * NU + L0, W = kMgTile + 2 * HU;
    const int ku = unit_of(t, (int)blockIdx.x);
    const Inst &I = insts[t.id[ku]];
    if (I.F[F_DONE]) return;
    const int lb = (int)blockIdx.x - t.boff[ku];
    const int ti = lb / t.bx[ku], tj = lb - ti * t.bx[ku];
    const LevelDev F = I.lev[level], Cc = I.lev[level + 1];
    const int i0 = ti * kMgTile, j0 = tj * kMgTile;
    __shared__ float su[W * W], sg[W * W], sc[W * W];
    __shared__ uint8_t sf[W * W];
    const float *gsrc = (L0 && par) ? I.cg_r1 : F.g;
    mg_stage<W>(F, F.uo, gsrc, I.g.px, I.g.py, i0 - HU, j0 - HU, su, sg, sf);
    __syncthreads();
    // red nodes: value plus the prolonged coarse correction (0 on fixed nodes)
    for (int k = threadIdx.x; k < W * W; k += kMgThreads) {
        const int a = k / W, c = k - a * W;
        int gi = i0 - HU + a, gj = j0 - HU + c;
        float v = 0.0f;
        if (((a + c) & 1) == 0 && !sf[k]) {
            if (I.g.px) gi = wrap_any(gi, F.NX);
            if (I.g.py) gj = wrap_any(gj, F.NY);
            v = su[k] + prolong_red(Cc.u, Cc.NX, Cc.NY, gi, gj);
        }
        sc[k] = v;
    }
    __syncthreads();
    // black update over window rows/cols 1 .. W-2 from the corrected reds
    for (int k = threadIdx.x; k < W * W; k += kMgThreads) {
        const int a = k / W, c = k - a * W;
        if (a < 1 || a > W - 2 || c < 1 || c > W - 2 || sf[k]) continue;
        if (((a + c) & 1) != 1) continue;
        float s = sg[k];
        s += sc[k - W];
        s += sc[k + W];
        s += sc[k - 1];
        s += sc[k + 1];
        su[k] = s * 0.25f;
    }
    __syncthreads();
    constexpr int MEND = L0 ? 2 * NU + 1 : 2 * NU;
#pragma unroll
    for (int m = 2; m < MEND; m++) {
        win_sweep<W>(su, sg, sf, m, m & 1);               // even m: red, odd m: black
        __syncthreads();
    }
    if (!L0) {
        // last red half-sweep on the own tile; write both colours to u
        for (int k = threadIdx.x; k < kMgTile * kMgTile; k += kMgThreads) {
            const int a = k / kMgTile, c = k - a * kMgTile;
            const int gi = i0 + a, gj = j0 + c;
            if (gi >= F.NX || gj >= F.NY) continue;
            const int w = (a + HU) * W + (c + HU);
            float z = 0.0f;                               // fixed nodes carry no correction
            if (!sf[w]) {
                z = su[w];
                if (((gi + gj) & 1) == 0) z = win_gs<W>(su, sg, w);
            }
            F.u[(long long)gi * F.NY + gj] = z;
        }
        return;
    }
    // level 0: the last red sweep covered the tile and its ring; z = su
    // (0 on fixed nodes), w = A z with the neighbours in the order x-1, x+1,
    // y-1, y+1
    double rz = 0.0, wz = 0.0;
    for (int k = threadIdx.x; k < kMgTile * kMgTile; k += kMgThreads) {
        const int a = k / kMgTile, c = k - a * kMgTile;
        const int gi = i0 + a, gj = j0 + c;
        if (gi >= F.NX || gj >= F.NY) continue;
        const long long n = (long long)gi * F.NY + gj;
        const int w = (a + HU) * W + (c + HU);
        float z = 0.0f, wv = 0.0f;
        if (!sf[w]) {
            z = su[w];
            float q = 4.0f * z;
            q -= su[w - W];
            q -= su[w + W];
            q -= su[w - 1];
            q -= su[w + 1];
            wv = q;
            rz += (double)sg[w] * (double)z;
            wz += (double)wv * (double)z;
        }
        F.u[n] = z;
        I.cg_w[n] = wv;
    }
    double v[2] = {rz, wz};
    block_partials<2>(v, pt);
}

constexpr int kMgSmooth = 1;     // pre- and post-smoothing steps on the fine levels

// The level-0 up kernel's r.z and (A z).z partials: a range of their own
// after the two the other reductions use, so that they survive until the
// next level-0 down kernel reads them (plain-CG instances of a batch reduce
// in between).
static Part cg_dot_part(Part pt) { return Part{pt.p + 2 * (size_t)pt.stride, pt.stride}; }

void launch_mg_down(const Inst *I, const Tab &t, int level, int mode, int par, Part pt, hipStream_t s)
{
    if (!t.n) return;
    const dim3 g(tab_blocks(t)), b(kMgThreads);
    const Part pq = cg_dot_part(pt);
    if (mode == 0) {
        hipLaunchKernelGGL((k_mg_down<kMgSmooth, 0>), g, b, 0, s, I, t, level, par, pt, pq);
    } else if (mode == 1) {
        hipLaunchKernelGGL((k_mg_down<kMgSmooth, 1>), g, b, 0, s, I, t, level, par, pt, pq);
        finalize(I, t, pt, OP_INIT, s);
    } else {
        // mode 3: the coarse kernel reduces the partials (fused update)
        hipLaunchKernelGGL((k_mg_down<kMgSmooth, 2>), g, b, 0, s, I, t, level, par, pt, pq);
        if (mode == 2) finalize(I, t, pt, OP_UPDATE, s);
    }
}

void launch_mg_up(const Inst *I, const Tab &t, int level, int par, Part pt, hipStream_t s)
{
    if (!t.n) return;
    const dim3 g(tab_blocks(t)), b(kMgThreads);
    if (level == 0) {
        // the next level-0 down kernel turns the partials into alpha and beta
        hipLaunchKernelGGL((k_mg_up<kMgSmooth, 1>), g, b, 0, s, I, t, level, par, cg_dot_part(pt));
    } else {
        hipLaunchKernelGGL((k_mg_up<kMgSmooth, 0>), g, b, 0, s, I, t, level, par, pt);
    }
}

// ---------------------------------------------------------------------------
// two fine levels l and l + 1 in one launch (one pre- / post-smoothing step):
// one 1024-thread block per 32 x 32 tile of level l + 1.  The block
// recomputes level l on the wider window its level-(l+1) window needs, so no
// block depends on another between the two levels.  Level l + 1's final
// correction is consumed inside the up kernel and never stored.
// ---------------------------------------------------------------------------

constexpr int kPairThreads = 1024;
constexpr int kPairDnF = 79;      // down, level l:     rows 2 I0 - 9 .. 2 I0 + 69
constexpr int kPairDnC = 37;      // down, level l + 1: rows I0 - 3 .. I0 + 33
constexpr int kPairUpC = 39;      // up, level l + 1:   rows I0 - 3 .. I0 + 35
constexpr int kPairUpF = 68;      // up, level l:       rows 2 I0 - 2 .. 2 I0 + 65

__host__ __device__ constexpr int pad16(int b) { return (b + 15) & ~15; }
__host__ __device__ constexpr int win_lds(int W) { return pad16(3 * W * W * 4) + pad16(W * W); }
constexpr int kPairDnLds = win_lds(kPairDnF) + win_lds(kPairDnC);
constexpr int kPairUpLds = win_lds(kPairUpC) + win_lds(kPairUpF);

// Window arrays at byte offset off: u, g, scratch (float) and the mask.
struct WinLds {
    float *u, *g, *r;
    uint8_t *f;
};
__device__ __forceinline__ WinLds win_at(unsigned char *lds, int off, int W)
{
    WinLds w;
    w.u = (float *)(lds + off);
    w.g = w.u + W * W;
    w.r = w.g + W * W;
    w.f = (uint8_t *)(lds + off + pad16(3 * W * W * 4));
    return w;
}

// Down half-cycles of levels l and l + 1: black half-sweep of level l from
// its red-from-zero start, level l's pre-smoothed tile nodes to uo, the
// restriction of its red residuals to the level-(l+1) window (g of the own
// tile stored), black half-sweep there, level l+1's tile to uo, and the
// restriction to level l + 2 (g and its red-from-zero start u).
__global__ __launch_bounds__(kPairThreads) void k_mg_down_pair(const Inst *insts, Tab t, int level)
{
    constexpr int WF = kPairDnF, WC = kPairDnC, NT = kPairThreads;
    extern __shared__ __align__(16) unsigned char lds[];
    const int ku = unit_of(t, (int)blockIdx.x);
    const Inst &I = insts[t.id[ku]];
    if (I.F[F_DONE]) return;
    const int lb = (int)blockIdx.x - t.boff[ku];
    const int ti = lb / t.bx[ku], tj = lb - ti * t.bx[ku];
    const LevelDev F = I.lev[level], C = I.lev[level + 1], N = I.lev[level + 2];
    const int px = I.g.px, py = I.g.py;
    const int I0 = ti * kMgTile, J0 = tj * kMgTile;
    const WinLds f = win_at(lds, 0, WF), c = win_at(lds, win_lds(WF), WC);
    const int tid = threadIdx.x;
    mg_stage<WF, NT>(F, F.u, F.g, px, py, 2 * I0 - 9, 2 * J0 - 9, f.u, f.g, f.f);
    for (int k = tid; k < WC * WC; k += NT) {
        const int a = k / WC, b = k - a * WC;
        const long long n = win_node(C.NX, C.NY, px, py, I0 - 3 + a, J0 - 3 + b);
        c.f[k] = n >= 0 ? C.fix[n] : 1;
    }
    __syncthreads();
    win_sweep<WF, NT>(f.u, f.g, f.f, 1, 1);               // black, rows 1 .. WF-2
    __syncthreads();
    for (int k = tid; k < 64 * 64; k += NT) {             // own level-l nodes
        const int a = k >> 6, b = k & 63;
        const int gi = 2 * I0 + a, gj = 2 * J0 + b;
        if (gi < F.NX && gj < F.NY) F.uo[(long long)gi * F.NY + gj] = f.u[(a + 9) * WF + (b + 9)];
    }
    for (int k = tid; k < WF * WF; k += NT) {             // red residuals, rows 2 .. WF-3
        const int a = k / WF, b = k - a * WF;
        if (a < 2 || a > WF - 3 || b < 2 || b > WF - 3 || ((a + b) & 1)) continue;
        float r = 0.0f;
        if (!f.f[k]) {
            float q = 4.0f * f.u[k];
            q -= f.u[k - WF];
            q -= f.u[k + WF];
            q -= f.u[k - 1];
            q -= f.u[k + 1];
            r = f.g[k] - q;
        }
        f.r[k] = r;
    }
    __syncthreads();
    for (int k = tid; k < WC * WC; k += NT) {             // restriction to the level-(l+1) window
        const int a = k / WC, b = k - a * WC;
        float gv = 0.0f, uv = 0.0f;
        if (!c.f[k]) {
            const int m = (3 + 2 * a) * WF + (3 + 2 * b);
            float acc = 0.0f;
            acc += 0.25f * f.r[m - WF - 1];
            acc += 0.25f * f.r[m - WF + 1];
            acc += 1.0f * f.r[m];
            acc += 0.25f * f.r[m + WF - 1];
            acc += 0.25f * f.r[m + WF + 1];
            gv = acc;
            if (((a + b) & 1) == 0) uv = gv * 0.25f;
        }
        c.g[k] = gv;
        c.u[k] = uv;
        const int gi = I0 - 3 + a, gj = J0 - 3 + b;
        if (a >= 3 && a < 35 && b >= 3 && b < 35 && gi < C.NX && gj < C.NY) C.g[(long long)gi * C.NY + gj] = gv;
    }
    __syncthreads();
    win_sweep<WC, NT>(c.u, c.g, c.f, 1, 1);               // black, rows 1 .. WC-2
    __syncthreads();
    for (int k = tid; k < kMgTile * kMgTile; k += NT) {   // own level-(l+1) nodes
        const int a = k / kMgTile, b = k - a * kMgTile;
        const int gi = I0 + a, gj = J0 + b;
        if (gi < C.NX && gj < C.NY) C.uo[(long long)gi * C.NY + gj] = c.u[(a + 3) * WC + (b + 3)];
    }
    for (int k = tid; k < WC * WC; k += NT) {             // red residuals, rows 2 .. WC-3
        const int a = k / WC, b = k - a * WC;
        if (a < 2 || a > WC - 3 || b < 2 || b > WC - 3 || ((a + b) & 1)) continue;
        float r = 0.0f;
        if (!c.f[k]) {
            float q = 4.0f * c.u[k];
            q -= c.u[k - WC];
            q -= c.u[k + WC];
            q -= c.u[k - 1];
            q -= c.u[k + 1];
            r = c.g[k] - q;
        }
        c.r[k] = r;
    }
    __syncthreads();
    if (tid < 256) {                                      // restriction to level l + 2
        const int ci = tid >> 4, cj = tid & 15;
        const int CI = (I0 >> 1) + ci, CJ = (J0 >> 1) + cj;
        if (CI < N.NX && CJ < N.NY) {
            const long long n = (long long)CI * N.NY + CJ;
            float gv = 0.0f, uv = 0.0f;
            if (!N.fix[n]) {
                const int m = (3 + 2 * ci) * WC + (3 + 2 * cj);
                float acc = 0.0f;
                acc += 0.25f * c.r[m - WC - 1];
                acc += 0.25f * c.r[m - WC + 1];
                acc += 1.0f * c.r[m];
                acc += 0.25f * c.r[m + WC - 1];
                acc += 0.25f * c.r[m + WC + 1];
                gv = acc;
                if (((CI + CJ) & 1) == 0) uv = gv * 0.25f;
            }
            N.g[n] = gv;
            N.u[n] = uv;
        }
    }
}

// Up half-cycles of levels l + 1 and l: level l+1's pre-smoothed window plus
// the prolonged level-(l+2) correction at its reds, black update, red
// half-sweep (its final correction, in LDS); then level l likewise with the
// prolongation read from that LDS result; level l's tile to u.
__global__ __launch_bounds__(kPairThreads) void k_mg_up_pair(const Inst *insts, Tab t, int level)
{
    constexpr int WC = kPairUpC, WF = kPairUpF, NT = kPairThreads;
    extern __shared__ __align__(16) unsigned char lds[];
    const int ku = unit_of(t, (int)blockIdx.x);
    const Inst &I = insts[t.id[ku]];
    if (I.F[F_DONE]) return;
    const int lb = (int)blockIdx.x - t.boff[ku];
    const int ti = lb / t.bx[ku], tj = lb - ti * t.bx[ku];
    const LevelDev F = I.lev[level], C = I.lev[level + 1], N = I.lev[level + 2];
    const int px = I.g.px, py = I.g.py;
    const int I0 = ti * kMgTile, J0 = tj * kMgTile;
    const WinLds c = win_at(lds, 0, WC), f = win_at(lds, win_lds(WC), WF);
    const int tid = threadIdx.x;
    mg_stage<WC, NT>(C, C.uo, C.g, px, py, I0 - 3, J0 - 3, c.u, c.g, c.f);
    mg_stage<WF, NT>(F, F.uo, F.g, px, py, 2 * I0 - 2, 2 * J0 - 2, f.u, f.g, f.f);
    __syncthreads();
    for (int k = tid; k < WC * WC; k += NT) {             // corrected reds of level l + 1
        const int a = k / WC, b = k - a * WC;
        float v = 0.0f;
        if (((a + b) & 1) == 0 && !c.f[k]) {
            int gi = I0 - 3 + a, gj = J0 - 3 + b;
            if (px) gi = wrap_any(gi, C.NX);
            if (py) gj = wrap_any(gj, C.NY);
            v = c.u[k] + prolong_red(N.u, N.NX, N.NY, gi, gj);
        }
        c.r[k] = v;
    }
    __syncthreads();
    for (int k = tid; k < WC * WC; k += NT) {             // black update, rows 1 .. WC-2
        const int a = k / WC, b = k - a * WC;
        if (a < 1 || a > WC - 2 || b < 1 || b > WC - 2 || c.f[k] || ((a + b) & 1) != 1) continue;
        float s = c.g[k];
        s += c.r[k - WC];
        s += c.r[k + WC];
        s += c.r[k - 1];
        s += c.r[k + 1];
        c.u[k] = s * 0.25f;
    }
    __syncthreads();
    win_sweep<WC, NT>(c.u, c.g, c.f, 2, 0);               // red, rows 2 .. WC-3
    __syncthreads();
    for (int k = tid; k < WF * WF; k += NT) {             // corrected reds of level l
        const int a = k / WF, b = k - a * WF;
        float v = 0.0f;
        if (((a + b) & 1) == 0 && !f.f[k]) {
            // level-(l+1) window row of fine row 2 I0 - 2 + a is 2 + (a >> 1)
            const int m = (2 + (a >> 1)) * WC + (2 + (b >> 1));
            float e;
            if (((a | b) & 1) == 0) e = c.u[m];
            else e = 0.25f * (c.u[m] + c.u[m + WC] + c.u[m + 1] + c.u[m + WC + 1]);
            v = f.u[k] + e;
        }
        f.r[k] = v;
    }
    __syncthreads();
    for (int k = tid; k < WF * WF; k += NT) {             // black update, rows 1 .. WF-2
        const int a = k / WF, b = k - a * WF;
        if (a < 1 || a > WF - 2 || b < 1 || b > WF - 2 || f.f[k] || ((a + b) & 1) != 1) continue;
        float s = f.g[k];
        s += f.r[k - WF];
        s += f.r[k + WF];
        s += f.r[k - 1];
        s += f.r[k + 1];
        f.u[k] = s * 0.25f;
    }
    __syncthreads();
    for (int k = tid; k < 64 * 64; k += NT) {             // red half-sweep of the own tile; tile to u
        const int a = k >> 6, b = k & 63;
        const int gi = 2 * I0 + a, gj = 2 * J0 + b;
        if (gi >= F.NX || gj >= F.NY) continue;
        const int w = (a + 2) * WF + (b + 2);
        float z = 0.0f;
        if (!f.f[w]) {
            z = f.u[w];
            if (((gi + gj) & 1) == 0) z = win_gs<WF>(f.u, f.g, w);
        }
        F.u[(long long)gi * F.NY + gj] = z;
    }
}

void launch_mg_pair(const Inst *I, const Tab &t, int level, bool down, hipStream_t s)
{
    if (!t.n) return;
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_mg_down_pair, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kPairDnLds);
        (void)hipFuncSetAttribute((const void *)k_mg_up_pair, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kPairUpLds);
        attr = true;
    }
    const dim3 g(tab_blocks(t)), b(kPairThreads);
    if (down) hipLaunchKernelGGL(k_mg_down_pair, g, b, kPairDnLds, s, I, t, level);
    else hipLaunchKernelGGL(k_mg_up_pair, g, b, kPairUpLds, s, I, t, level);
}

// ---------------------------------------------------------------------------
// coarse levels: the rest of the V-cycle in one work-group per instance,
// all in LDS
// ---------------------------------------------------------------------------

// Gauss-Seidel value from the four neighbours without mask tests: fixed
// nodes hold u = 0 on the LDS levels (staged as 0, never updated).  A free
// node never lies on a bounded edge, so only periodic axes wrap.
__device__ __forceinline__ float gs_nofix(const float *u, const float *gg, int i, int j, int NX, int NY)
{
    Nb b = nbs(i, j, NX, NY);
    float s = gg[i * NY + j];
    s += u[b.im * NY + j];
    s += u[b.ip * NY + j];
    s += u[i * NY + b.jm];
    s += u[i * NY + b.jp];
    return s * 0.25f;
}

// q / d for 0 <= q < 2^22 and d >= 1 from rcp = 1/d in float32: the exact
// quotient (q + 1/2) / d lies at least 1/(2d) from an integer, more than
// the rounding error of the product.
__device__ __forceinline__ int div_rcp(int q, float rcp) { return (int)(((float)q + 0.5f) * rcp); }

// Phases of the LDS levels.  Each is run by a group of threads (first,
// step): the whole work-group, or one wavefront for the small levels, with
// the group's barrier between phases.  Half-sweeps and the red-node passes
// visit the nodes of their colour only (j = 2 jj + ((i + colour) & 1)).
struct CLev {
    float *u, *g;
    const uint8_t *f;
    int NX, NY;
};

// Gauss-Seidel half-sweep of one colour (1 black, 0 red).
__device__ __forceinline__ void c_sweep(const CLev &L, int col, int first, int step)
{
    const int HW = (L.NY + 1) >> 1;
    const float rcp = 1.0f / (float)HW;
    for (int q = first; q < L.NX * HW; q += step) {
        const int i = div_rcp(q, rcp), j = 2 * (q - i * HW) + ((i + col) & 1);
        if (j < L.NY && !L.f[i * L.NY + j]) L.u[i * L.NY + j] = gs_nofix(L.u, L.g, i, j, L.NX, L.NY);
    }
}

// Residual g - A u at the red nodes into sr (0 at fixed nodes).
__device__ __forceinline__ void c_resid_red(const CLev &L, float *sr, int first, int step)
{
    const int HW = (L.NY + 1) >> 1, NY = L.NY;
    const float rcp = 1.0f / (float)HW;
    for (int q = first; q < L.NX * HW; q += step) {
        const int i = div_rcp(q, rcp), j = 2 * (q - i * HW) + (i & 1);
        if (j >= NY) continue;
        const int k = i * NY + j;
        float r = 0.0f;
        if (!L.f[k]) {
            Nb b = nbs(i, j, L.NX, NY);
            float v = 4.0f * L.u[k];
            v -= L.u[b.im * NY + j];
            v -= L.u[b.ip * NY + j];
            v -= L.u[i * NY + b.jm];
            v -= L.u[i * NY + b.jp];
            r = L.g[k] - v;
        }
        sr[k] = r;
    }
}

// Restriction of the red residuals sr of level L to level C (g), with C's
// red-from-zero start (u).
__device__ __forceinline__ void c_restrict(const CLev &L, const float *sr, const CLev &C, int px, int py,
                                           int first, int step)
{
    const int NX = L.NX, NY = L.NY;
    const float rcp = 1.0f / (float)C.NY;
    for (int k = first; k < C.NX * C.NY; k += step) {
        const int Ic = div_rcp(k, rcp), Jc = k - Ic * C.NY;
        float gv = 0.0f, uv = 0.0f;
        if (!C.f[k]) {
            float acc = 0.0f;
#pragma unroll
            for (int di = -1; di <= 1; di++) {
#pragma unroll
                for (int dj = -1; dj <= 1; dj++) {
                    if ((di + dj) & 1) continue;
                    int ai = 2 * Ic + di, cj = 2 * Jc + dj;
                    if (px) ai = wrap_hi(wrap_lo(ai, NX), NX);
                    else if (ai < 0 || ai >= NX) continue;
                    if (py) cj = wrap_hi(wrap_lo(cj, NY), NY);
                    else if (cj < 0 || cj >= NY) continue;
                    const float w = (di == 0) ? 1.0f : 0.25f;
                    acc += w * sr[ai * NY + cj];
                }
            }
            gv = acc;
            if (((Ic + Jc) & 1) == 0) uv = gv * 0.25f;
        }
        C.g[k] = gv;
        C.u[k] = uv;
    }
}

// Red nodes of level L plus the prolonged correction of level C into sr (0
// at fixed nodes).
__device__ __forceinline__ void c_correct_red(const CLev &L, const CLev &C, float *sr, int first, int step)
{
    const int HW = (L.NY + 1) >> 1, NY = L.NY;
    const float rcp = 1.0f / (float)HW;
    for (int q = first; q < L.NX * HW; q += step) {
        const int i = div_rcp(q, rcp), j = 2 * (q - i * HW) + (i & 1);
        if (j >= NY) continue;
        const int k = i * NY + j;
        sr[k] = L.f[k] ? 0.0f : L.u[k] + prolong_red(C.u, C.NX, C.NY, i, j);
    }
}

// Black update of level L from the corrected reds in sr.
__device__ __forceinline__ void c_black_from(const CLev &L, const float *sr, int first, int step)
{
    const int HW = (L.NY + 1) >> 1, NY = L.NY;
    const float rcp = 1.0f / (float)HW;
    for (int q = first; q < L.NX * HW; q += step) {
        const int i = div_rcp(q, rcp), j = 2 * (q - i * HW) + ((i + 1) & 1);
        if (j >= NY || L.f[i * NY + j]) continue;
        Nb b = nbs(i, j, L.NX, NY);
        float v = L.g[i * NY + j];
        v += sr[b.im * NY + j];
        v += sr[b.ip * NY + j];
        v += sr[i * NY + b.jm];
        v += sr[i * NY + b.jp];
        L.u[i * NY + j] = v * 0.25f;
    }
}

// One wavefront's barrier: its lanes run in lockstep and LDS serves one
// wavefront's accesses in order, so fences around a wave barrier order the
// phases.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int kCoarseWaveNodes = 200;   // LDS levels at most this size are run by one wavefront

// Sums of four floats over the 64 lanes of a wavefront (all lanes active),
// returned in lane 63: row-local butterflies (quad permutes, row mirrors)
// give every lane its row sum, then two row broadcasts carry the sums of
// rows 0-2 up to row 3.  A fixed order of additions.
#define DPPF_STEP(ctrl, rmask)                                                                          \
    a += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), ctrl, rmask, 0xF, false));    \
    b += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(b), ctrl, rmask, 0xF, false));    \
    c += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(c), ctrl, rmask, 0xF, false));    \
    d += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(d), ctrl, rmask, 0xF, false));
__device__ __forceinline__ void wave_sum4_f32(float &a, float &b, float &c, float &d)
{
    DPPF_STEP(0xB1, 0xF)   // quad_perm [1,0,3,2]
    DPPF_STEP(0x4E, 0xF)   // quad_perm [2,3,0,1]
    DPPF_STEP(0x141, 0xF)  // row_half_mirror
    DPPF_STEP(0x140, 0xF)  // row_mirror
    DPPF_STEP(0x142, 0xA)  // row_bcast:15 into rows 1, 3
    DPPF_STEP(0x143, 0xC)  // row_bcast:31 into rows 2, 3
}
#undef DPPF_STEP

// Exact solve of the coarsest level, u = A^-1 g, from the packed lower
// triangle T of the inverse the host factorised (row r: columns 0 .. r padded
// to a multiple of 4, diagonal halved, zero rows and columns at fixed nodes).
// Wavefront w takes rows w, w + 16, ...; its lanes read 16-byte pieces of the
// row (Q pieces per lane and row), R rows per pass with every load of a pass
// issued before any is used.  Each stored entry serves twice: its row's dot
// product with g (the lower part of u[r] and half its diagonal term, summed
// across the wave) and T[r][c] g[r] added to the lane's partial sum for
// column c (the upper part and the other half).  The column partials of the
// 16 wavefronts meet in LDS (part, 16 x n floats) and are summed in a fixed
// order.  Every stored float is read once.  Small levels (n <= 256: one piece
// per lane and row, 8 rows of a wave per pass) pay one or two memory latencies.
template <int Q, int R>
__device__ __forceinline__ void c_dense(const CLev &L, const float *__restrict__ T, int n, float *part, int tid)
{
    static_assert(R == 2 || R % 4 == 0, "rows per pass: 2 or a multiple of 4 (four-way wave sums)");
    const int lane = tid & 63, w = tid >> 6;
    const int npc = (n + 3) >> 2;                 // 16-byte pieces of the longest row
    // g is read in 16-byte pieces: its padding up to a multiple of 4 (inside
    // the level's 16-byte rounded array) is cleared first
    if (tid < 4 && n + tid < 4 * npc) L.g[n + tid] = 0.0f;
    __syncthreads();
    const float4 *g4 = (const float4 *)L.g;
    float4 acc[Q];
#pragma unroll
    for (int q = 0; q < Q; q++) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int r0 = w; r0 < n; r0 += R * kCoarseWaves) {
        float4 t[R][Q];
#pragma unroll
        for (int i = 0; i < R; i++) {
            const int r = r0 + i * kCoarseWaves;
            const int len = r < n ? (r >> 2) + 1 : 0;      // pieces of row r
            const float4 *row = (const float4 *)(T + tri_off(r < n ? r : 0));
#pragma unroll
            for (int q = 0; q < Q; q++) {
                const int k = lane + 64 * q;
                t[i][q] = k < len ? row[k] : make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        float4 gq[Q];
#pragma unroll
        for (int q = 0; q < Q; q++) {
            const int k = lane + 64 * q;
            gq[q] = k < npc ? g4[k] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        float dot[R];
#pragma unroll
        for (int i = 0; i < R; i++) {
            const int r = r0 + i * kCoarseWaves;
            const float gr = r < n ? L.g[r] : 0.0f;
            dot[i] = 0.0f;
#pragma unroll
            for (int q = 0; q < Q; q++) {
                dot[i] += t[i][q].x * gq[q].x + t[i][q].y * gq[q].y + t[i][q].z * gq[q].z + t[i][q].w * gq[q].w;
                acc[q].x += t[i][q].x * gr;
                acc[q].y += t[i][q].y * gr;
                acc[q].z += t[i][q].z * gr;
                acc[q].w += t[i][q].w * gr;
            }
        }
        if constexpr (R == 2) {
            float d2 = 0.0f, d3 = 0.0f;
            wave_sum4_f32(dot[0], dot[1], d2, d3);
        } else {
#pragma unroll
            for (int i = 0; i < R; i += 4) wave_sum4_f32(dot[i], dot[i + 1], dot[i + 2], dot[i + 3]);
        }
        if (lane == 63) {
#pragma unroll
            for (int i = 0; i < R; i++) {
                const int r = r0 + i * kCoarseWaves;
                if (r < n) L.u[r] = dot[i];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Q; q++) {
        const int k = lane + 64 * q, c = 4 * k;
        if (k < npc) {
            float *pw = part + (size_t)w * n;
            if (c < n) pw[c] = acc[q].x;
            if (c + 1 < n) pw[c + 1] = acc[q].y;
            if (c + 2 < n) pw[c + 2] = acc[q].z;
            if (c + 3 < n) pw[c + 3] = acc[q].w;
        }
    }
    __syncthreads();
    for (int c = tid; c < n; c += 64 * kCoarseWaves) {
        float v = L.u[c];
#pragma unroll
        for (int q = 0; q < kCoarseWaves; q++) v += part[(size_t)q * n + c];
        L.u[c] = v;
    }
}

constexpr int kDenseOnePass = 256;   // coarsest levels up to this size: one piece per lane, 8 rows per pass

__device__ __forceinline__ void c_dense_any(const CLev &L, const float *__restrict__ T, int n, float *part, int tid)
{
    if (n <= kDenseOnePass) c_dense<1, 8>(L, T, n, part, tid);
    else c_dense<(kDenseMaxNodes + 255) / 256, 2>(L, T, n, part, tid);
}

constexpr int kCoarsePre = 4;   // 16-byte pieces per thread loaded before the level-0 reduction (fetch calls)

// The levels from lg on: one 1024-thread work-group per instance, every level
// in LDS.  Per level on the way down a black half-sweep, the red residuals,
// their restriction to the next level with its red-from-zero start; on the
// coarsest level red-black sweeps; per level on the way up the corrected
// reds, the black update from them, then a red half-sweep.  The levels of at
// most kCoarseWaveNodes nodes, from the first such level to the coarsest and
// back, are run by the first wavefront alone (no work-group barriers).
// With fuse set it first does what k_finalize(OP_UPDATE) does after the
// level-0 CG step (t0: that launch's units, in the same order as t): the
// totals of its partials in the same order, the iteration count and the
// inner stop test; one launch fewer per iteration.  The paired or single
// fine levels between the two run on regardless (their output is then
// unused).
__global__ __launch_bounds__(1024) void k_coarse(const Inst *insts, Tab t, Tab t0, Part pt, int fuse)
{
    const Inst &I = insts[t.id[blockIdx.x]];
    const int tid = threadIdx.x, nt = blockDim.x;
    if (!fuse && I.F[F_DONE]) return;
    const CoarseArgs &a = I.coarse;
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int tab[3][kMaxLev];
    __shared__ int dims[2][kMaxLev];
    // 16-byte pieces to stage: the masks of every level, then the first
    // level's g (the global arrays are 256-byte aligned and padded, the LDS
    // ones 16-byte rounded, so whole pieces stay inside both)
    __shared__ const unsigned char *src[kMaxLev + 1];
    __shared__ int dst[kMaxLev + 1], cum[kMaxLev + 2];
    if (tid == 0) {
        int c = 0;
        for (int l = 0; l < a.nlev; l++) {
            tab[0][l] = a.off_u[l];
            tab[1][l] = a.off_g[l];
            tab[2][l] = a.off_f[l];
            dims[0][l] = a.NX[l];
            dims[1][l] = a.NY[l];
            src[l] = a.fix[l];
            dst[l] = a.off_f[l];
            cum[l] = c;
            c += (a.NX[l] * a.NY[l] + 15) >> 4;
        }
        src[a.nlev] = (const unsigned char *)a.g_top;
        dst[a.nlev] = a.off_g[0];
        cum[a.nlev] = c;
        cum[a.nlev + 1] = c + ((a.NX[0] * a.NY[0] + 3) >> 2);
    }
    __syncthreads();
    const int nlev = a.nlev, px = a.px, py = a.py, npieces = cum[nlev + 1];
    // every thread issues its first pieces' loads before the level-0
    // reduction below, so their latencies overlap
    auto fetch = [&](int m, uint4 &v, int &d) {
        const int p = tid + m * nt;
        d = -1;
        if (p < npieces) {
            int k = 0;
            while (p >= cum[k + 1]) k++;
            const int q = p - cum[k];
            v = ((const uint4 *)src[k])[q];
            d = dst[k] + 16 * q;
        }
    };
    uint4 pv0, pv1, pv2, pv3;
    int pd0, pd1, pd2, pd3;
    fetch(0, pv0, pd0);
    fetch(1, pv1, pd1);
    fetch(2, pv2, pd2);
    fetch(3, pv3, pd3);
    if (fuse) {
        // what k_finalize(OP_UPDATE) does after the level-0 CG step (t0: that
        // launch's units, in the same order as t): the totals of its partials
        // in the same order, the iteration count and the inner stop test
        __shared__ double fsh[2][4];
        __shared__ int fdone;
        if (tid == 256) {
            // a wavefront outside the sums reads the scalars and flags the
            // update uses (just written by other kernels, on other XCDs), so
            // that thread 0 finds them in the caches after the barrier (the
            // empty asm keeps the loads)
            const double *ws = I.S;
            const int *wf = I.F;
            const double warm = ws[S_ETA2] + ws[S_RR0] + ws[S_CG_NALPHA] + ws[S_CG_NBETA] + ws[S_CG_NGAMMA] +
                                (double)(wf[F_ITER] + wf[F_ITER_TOT] + wf[F_PASSES]);
            asm volatile("" ::"v"(warm));
        }
        partial_sums_256(pt, t0.boff[blockIdx.x], t0.boff[blockIdx.x + 1], 2, fsh, tid);
        __syncthreads();
        if (tid == 0) {
            apply_op(I, OP_UPDATE, fsh[0][0] + fsh[0][1] + fsh[0][2] + fsh[0][3],
                     fsh[1][0] + fsh[1][1] + fsh[1][2] + fsh[1][3]);
            fdone = I.F[F_DONE];
        }
        __syncthreads();
        if (fdone) return;
    }
    if (pd0 >= 0) *(uint4 *)(lds + pd0) = pv0;
    if (pd1 >= 0) *(uint4 *)(lds + pd1) = pv1;
    if (pd2 >= 0) *(uint4 *)(lds + pd2) = pv2;
    if (pd3 >= 0) *(uint4 *)(lds + pd3) = pv3;
    for (int p = tid + kCoarsePre * nt; p < npieces; p += nt) {
        int k = 0;
        while (p >= cum[k + 1]) k++;
        const int q = p - cum[k];
        *(uint4 *)(lds + dst[k] + 16 * q) = ((const uint4 *)src[k])[q];
    }
    auto lev = [&](int l) {
        CLev L;
        L.u = (float *)(lds + tab[0][l]);
        L.g = (float *)(lds + tab[1][l]);
        L.f = (const uint8_t *)(lds + tab[2][l]);
        L.NX = dims[0][l];
        L.NY = dims[1][l];
        return L;
    };
    float *sr = (float *)(lds + a.off_s);
    __syncthreads();
    {
        const CLev L = lev(0);
        const int N = L.NX * L.NY;
        const float rcp = 1.0f / (float)L.NY;
        for (int k = tid; k < N; k += nt) {
            const int i = div_rcp(k, rcp), j = k - i * L.NY;
            L.u[k] = (!L.f[k] && ((i + j) & 1) == 0) ? L.g[k] * 0.25f : 0.0f;
        }
    }
    __syncthreads();
    // first level run by one wavefront (nlev when none is small enough)
    int ls = 0;
    while (ls < nlev && dims[0][ls] * dims[1][ls] > kCoarseWaveNodes) ls++;
    const int lb = ls < nlev - 1 ? ls : nlev - 1;           // levels below lb descend with the work-group
    for (int l = 0; l < lb; l++) {
        const CLev L = lev(l), C = lev(l + 1);
        c_sweep(L, 1, tid, nt);
        __syncthreads();
        c_resid_red(L, sr, tid, nt);
        __syncthreads();
        c_restrict(L, sr, C, px, py, tid, nt);
        __syncthreads();
    }
    if (ls < nlev) {
        if (tid < 64) {
            for (int l = ls; l < nlev - 1; l++) {
                const CLev L = lev(l), C = lev(l + 1);
                c_sweep(L, 1, tid, 64);
                wave_sync();
                c_resid_red(L, sr, tid, 64);
                wave_sync();
                c_restrict(L, sr, C, px, py, tid, 64);
                wave_sync();
            }
        }
        if (a.dense_n) {
            __syncthreads();
            c_dense_any(lev(nlev - 1), a.ainv, a.dense_n, (float *)(lds + a.off_p), tid);
            __syncthreads();
        }
        if (tid < 64) {
            if (!a.dense_n) {
                // coarsest: red-black sweeps (the first black completes the pre-smoothing)
                const CLev L = lev(nlev - 1);
                for (int sw = 0; sw < a.sweeps; sw++) {
                    c_sweep(L, 1, tid, 64);
                    wave_sync();
                    c_sweep(L, 0, tid, 64);
                    wave_sync();
                }
            }
            for (int l = nlev - 2; l >= ls; l--) {
                const CLev F = lev(l), C = lev(l + 1);
                c_correct_red(F, C, sr, tid, 64);
                wave_sync();
                c_black_from(F, sr, tid, 64);
                wave_sync();
                c_sweep(F, 0, tid, 64);
                wave_sync();
            }
        }
        __syncthreads();
    } else if (a.dense_n) {
        c_dense_any(lev(nlev - 1), a.ainv, a.dense_n, (float *)(lds + a.off_p), tid);
        __syncthreads();
    } else {
        const CLev L = lev(nlev - 1);
        for (int sw = 0; sw < a.sweeps; sw++) {
            c_sweep(L, 1, tid, nt);
            __syncthreads();
            c_sweep(L, 0, tid, nt);
            __syncthreads();
        }
    }
    for (int l = lb - 1; l >= 0; l--) {
        const CLev F = lev(l), C = lev(l + 1);
        c_correct_red(F, C, sr, tid, nt);
        __syncthreads();
        c_black_from(F, sr, tid, nt);
        __syncthreads();
        c_sweep(F, 0, tid, nt);
        __syncthreads();
    }
    {
        const int N = dims[0][0] * dims[1][0];
        const float *u0 = (const float *)(lds + tab[0][0]);
        for (int k = tid; k < N; k += nt) a.u_top[k] = u0[k];
    }
}

void launch_coarse(const Inst *I, const Tab &t, int lds_bytes, const Tab &t0, Part pt, bool fuse, hipStream_t s)
{
    if (!t.n) return;
    static int allowed = 64 * 1024;
    if (lds_bytes > allowed) {
        (void)hipFuncSetAttribute((const void *)k_coarse, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
        allowed = lds_bytes;
    }
    hipLaunchKernelGGL(k_coarse, dim3(t.n), dim3(1024), lds_bytes, s, I, t, t0, pt, fuse ? 1 : 0);
}

// ---------------------------------------------------------------------------
// particles: gather, leapfrog push, wall test, deposit (eqs. 1-4)
// ---------------------------------------------------------------------------

// Sums of four 32-bit values over the 64 lanes (all lanes active), returned
// as wave-uniform values.  Row-local butterflies (quad permutes, row
// mirrors) give every lane its row sum, then two row broadcasts carry the
// sums of rows 0-2 upward to lane 63.  The four chains are interleaved so
// the DPP read-after-write wait states are filled with useful work.
#define DPP_STEP(ctrl, rmask)                                                                  \
    a += (unsigned)__builtin_amdgcn_update_dpp(0, (int)a, ctrl, rmask, 0xF, false);            \
    b += (unsigned)__builtin_amdgcn_update_dpp(0, (int)b, ctrl, rmask, 0xF, false);            \
    c += (unsigned)__builtin_amdgcn_update_dpp(0, (int)c, ctrl, rmask, 0xF, false);            \
    d += (unsigned)__builtin_amdgcn_update_dpp(0, (int)d, ctrl, rmask, 0xF, false);
__device__ __forceinline__ void wave_sum4_u32(unsigned &a, unsigned &b, unsigned &c, unsigned &d)
{
    DPP_STEP(0xB1, 0xF)   // quad_perm [1,0,3,2]
    DPP_STEP(0x4E, 0xF)   // quad_perm [2,3,0,1]
    DPP_STEP(0x141, 0xF)  // row_half_mirror
    DPP_STEP(0x140, 0xF)  // row_mirror
    DPP_STEP(0x142, 0xA)  // row_bcast:15 into rows 1, 3
    DPP_STEP(0x143, 0xC)  // row_bcast:31 into rows 2, 3
    a = (unsigned)__builtin_amdgcn_readlane((int)a, 63);
    b = (unsigned)__builtin_amdgcn_readlane((int)b, 63);
    c = (unsigned)__builtin_amdgcn_readlane((int)c, 63);
    d = (unsigned)__builtin_amdgcn_readlane((int)d, 63);
}
#undef DPP_STEP

// Arguments of the particle kernels resolved once per block into plain
// scalars and pointers (the storage set in use is device info[7], flipped
// by every re-binning), so particle stores cannot force them to be reloaded.
// Global-memory (address space 1) pointers: loads, stores and atomics on
// them compile to global_* instructions, which do not share the LDS wait
// counter the way flat accesses do, so the deposit's LDS atomics never wait
// for outstanding particle loads.
#define GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ GLOBAL T *to_global(T *p) { return (GLOBAL T *)p; }
typedef int nt_i4 __attribute__((ext_vector_type(4)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_f4(GLOBAL const float4 *p)
{
    const nt_f4 v = *(GLOBAL const nt_f4 *)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void gatomic_add(GLOBAL unsigned long long *p, unsigned long long v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct PK {
    Geom g;
    int TX, TY, H, WX, WY, tiles_y;
    GLOBAL const uint8_t *cell_cond;
    GLOBAL const float4 *E4;
    GLOBAL int32_t *cell;
    GLOBAL float *ox, *oy, *vx, *vy;
    GLOBAL unsigned long long *rho;
    float qdt, dtf, hq;
    int box_i_top, box_j_lo, box_j_hi, species;
    GLOBAL unsigned long long *surf;
    GLOBAL unsigned long long *iad;
    HitLog log;
    const long long *step;
    // LDS copy of the conductor map of cells c0i .. c0i+CW-1, c0j .. c0j+CH-1
    // (the block's deposit window and a one-cell frame; CW = 0: none)
    const uint8_t *scc;
    int c0i, c0j, CW, CH;
    // the same origin taken into [0, n) on a periodic axis, and the wrap
    // length of each axis (n when periodic, 0 when bounded)
    int c0wi, c0wj, nwx, nwy;
};

__device__ __forceinline__ PK resolve(const PushArgs &a)
{
    PK k;
    k.scc = nullptr;
    k.c0i = k.c0j = k.CW = k.CH = 0;
    k.c0wi = k.c0wj = k.nwx = k.nwy = 0;
    const int set = (int)a.info[7];
    k.g = a.g;
    k.TX = a.TX;
    k.TY = a.TY;
    k.H = a.H;
    k.WX = a.WX;
    k.WY = a.WY;
    k.tiles_y = a.tiles_y;
    k.cell_cond = to_global(a.cell_cond);
    k.E4 = to_global(a.E4);
    k.cell = to_global(set ? a.cell[1] : a.cell[0]);
    k.ox = to_global(set ? a.ox[1] : a.ox[0]);
    k.oy = to_global(set ? a.oy[1] : a.oy[0]);
    k.vx = to_global(set ? a.vx[1] : a.vx[0]);
    k.vy = to_global(set ? a.vy[1] : a.vy[0]);
    k.rho = to_global(a.rho);
    k.qdt = a.qdt;
    k.dtf = a.dtf;
    k.hq = a.hq;
    k.box_i_top = a.box_i_top;
    k.box_j_lo = a.box_j_lo;
    k.box_j_hi = a.box_j_hi;
    k.species = a.species;
    k.surf = to_global(a.surf);
    k.iad = to_global(a.iad);
    k.log = a.log;
    k.step = a.step;
    return k;
}

// Cell-by-cell walk of the straight segment (Dx, Dy) from offsets (x0, y0)
// in cell (ci, cj) across sx, sy faces (not both 0): the earlier face first,
// compared as (fx + kx)|Dy| <= (fy + ky)|Dx| (ties cross x).  Stops at the
// first cell outside a bounded axis or inside a conductor: dead = direction
// (0 +x, 1 -x, 2 +y, 3 -y) + 4 when the last cell occupied (ei, ej) lies in the
// trench box; else dead stays -1 and (ei, ej) is the final cell.
__device__ __forceinline__ void walk_cells(const PK &a, float x0, float y0, float Dx, float Dy, int sx, int sy,
                                           int &dead, int &ei, int &ej)
{
    const Geom &g = a.g;
    const float ax = fabsf(Dx), ay = fabsf(Dy);
    const float fx = sx > 0 ? 1.0f - x0 : x0, fy = sy > 0 ? 1.0f - y0 : y0;
    const int nxs = abs(sx), nys = abs(sy);
    const int di = sx > 0 ? 1 : -1, dj = sy > 0 ? 1 : -1;
    int kx = 0, ky = 0;
    while (kx < nxs || ky < nys) {
        bool gox;
        if (ky >= nys) gox = true;
        else if (kx >= nxs) gox = false;
        else gox = ((fx + (float)kx) * ay <= (fy + (float)ky) * ax);
        int ni = ei, nj = ej, dir;
        if (gox) { ni = ei + di; kx++; dir = di > 0 ? 0 : 1; }
        else { nj = ej + dj; ky++; dir = dj > 0 ? 2 : 3; }
        bool out = false;
        if (g.px) ni = wrap_hi(wrap_lo(ni, g.nx), g.nx);
        else if (ni < 0 || ni >= g.nx) out = true;
        if (g.py) nj = wrap_hi(wrap_lo(nj, g.ny), g.ny);
        else if (nj < 0 || nj >= g.ny) out = true;
        if (!out) {
            // conductor test from the block's LDS map when the cell lies in it
            int li = ni - a.c0i, lj = nj - a.c0j;
            if (g.px) { if (li < 0) li += g.nx; else if (li >= g.nx) li -= g.nx; }
            if (g.py) { if (lj < 0) lj += g.ny; else if (lj >= g.ny) lj -= g.ny; }
            const bool loc = li >= 0 && li < a.CW && lj >= 0 && lj < a.CH;
            if (loc ? a.scc[li * a.CH + lj] : a.cell_cond[(long long)ni * g.ny + nj]) out = true;
        }
        if (out) {
            const bool inbox = ei >= a.box_i_top && ej >= a.box_j_lo && ej < a.box_j_hi;
            dead = dir + (inbox ? 4 : 0);
            break;
        }
        ei = ni;
        ej = nj;
    }
}

// Leapfrog push of one particle with the bilinear gather of its cell's
// corner fields and the cell-by-cell wall test (eqs. 1-4).  Computes the new
// velocity (ux, uy), offsets (nxo, nyo) and cell (ei, ej); returns false when
// the particle was removed (class in dead, last cell occupied in ei, ej).
__device__ __forceinline__ bool push_core(const PK &a, float x0, float y0, float vx0, float vy0,
                                          float4 ea, float4 eb, int ci, int cj, int &dead, int &ei,
                                          int &ej, float &ux, float &uy, float &nxo, float &nyo)
{
    const float wx0 = 1.0f - x0, wy0 = 1.0f - y0;
    const float w00 = wx0 * wy0, w10 = x0 * wy0, w01 = wx0 * y0, w11 = x0 * y0;
    float ex = w00 * ea.x;
    ex = ex + w10 * ea.z;
    ex = ex + w01 * eb.x;
    ex = ex + w11 * eb.z;
    float ey = w00 * ea.y;
    ey = ey + w10 * ea.w;
    ey = ey + w01 * eb.y;
    ey = ey + w11 * eb.w;
    ux = vx0 + a.qdt * ex;
    uy = vy0 + a.qdt * ey;
    const float Dx = ux * a.dtf, Dy = uy * a.dtf;
    const float x1 = x0 + Dx, y1 = y0 + Dy;
    const float fsx = floorf(x1), fsy = floorf(y1);
    dead = -1;
    ei = ci;
    ej = cj;
    int sx = 0, sy = 0;
    if (!(fabsf(fsx) < 1.0e6f && fabsf(fsy) < 1.0e6f)) {
        dead = 8;
    } else {
        sx = (int)fsx;
        sy = (int)fsy;
        if (sx != 0 || sy != 0) walk_cells(a, x0, y0, Dx, Dy, sx, sy, dead, ei, ej);
    }
    nxo = x0;
    nyo = y0;
    if (dead >= 0) return false;
    nxo = x1 - (float)sx;
    nyo = y1 - (float)sy;
    if (nxo >= 1.0f) nxo = 0x1.fffffep-1f;
    if (nyo >= 1.0f) nyo = 0x1.fffffep-1f;
    return true;
}

// ---- ion recycling (Sec. III.A, III.C) --------------------------------------
// A lost ion is replaced by a thermal ion in the bulk rows 0 .. rows-1, the
// ionisation of the ambient gas.  Counter-based generator Philox4x32-10
// (Salmon, Moraes, Dror and Shaw, SC 2011): ten rounds of two 32 x 32-bit
// products (multipliers 0xD2511F53, 0xCD9E8D57), the key bumped by the Weyl
// constants 0x9E3779B9, 0xBB67AE85 between rounds.  Counter (step, bits of
// the lost ion's v_x after the kick, bits of its offsets before the move),
// keys (k0, k1) and (k0, k1 + 1):
//   cell (r0 >> 8) * rows >> 24, (r1 >> 8) * ny >> 24; offsets (r2 >> 8), (r3 >> 8) * 2^-24;
//   velocity vth sqrt(-2 ln u) (cos, sin)(2 pi v), u = ((q0 >> 8) + 1) 2^-24,
//   v = (q1 >> 8) 2^-24, in double, rounded to float.
struct Philox4 {
    unsigned x, y, z, w;
};

__device__ __forceinline__ Philox4 philox4x32_10(unsigned c0, unsigned c1, unsigned c2, unsigned c3, unsigned k0,
                                                 unsigned k1)
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const unsigned lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const unsigned n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return Philox4{c0, c1, c2, c3};
}

struct NewIon {
    int ci, cj;
    float ox, oy, vx, vy;
};

__device__ __forceinline__ NewIon recycled_ion(unsigned long long step, float ux, float x0, float y0, unsigned k0,
                                               unsigned k1, int rows, int ny, double vth)
{
    const unsigned c0 = (unsigned)step, c1 = __float_as_uint(ux);
    const unsigned c2 = __float_as_uint(x0), c3 = __float_as_uint(y0);
    const Philox4 r = philox4x32_10(c0, c1, c2, c3, k0, k1);
    const Philox4 q = philox4x32_10(c0, c1, c2, c3, k0, k1 + 1u);
    NewIon n;
    n.ci = (int)(((unsigned long long)(r.x >> 8) * (unsigned)rows) >> 24);
    n.cj = (int)(((unsigned long long)(r.y >> 8) * (unsigned)ny) >> 24);
    n.ox = (float)(r.z >> 8) * 0x1p-24f;
    n.oy = (float)(r.w >> 8) * 0x1p-24f;
    const double u = (double)((q.x >> 8) + 1u) * 0x1p-24, v = (double)(q.y >> 8) * 0x1p-24;
    const double rad = sqrt(-2.0 * log(u)), ang = 6.283185307179586 * v;
    n.vx = (float)(vth * rad * cos(ang));
    n.vy = (float)(vth * rad * sin(ang));
    return n;
}

// push_core plus the particle's stores (velocity always; offsets if it
// stays; the cell code when it changes or the particle is removed).
__device__ __forceinline__ bool push_particle(const PK &a, int p, int c, float &x0, float &y0,
                                              float vx0, float vy0, float4 ea, float4 eb, int &ci,
                                              int &cj, int &dead, int &ei, int &ej, float &ux,
                                              float &uy)
{
    float nxo, nyo;
    const bool alive = push_core(a, x0, y0, vx0, vy0, ea, eb, ci, cj, dead, ei, ej, ux, uy, nxo, nyo);
    a.vx[p] = ux;
    a.vy[p] = uy;
    if (!alive) {
        a.cell[p] = -1 - dead;
        return false;
    }
    a.ox[p] = nxo;
    a.oy[p] = nyo;
    const int nc = (int)(((unsigned)ei << 16) | (unsigned)ej);
    if (nc != c) a.cell[p] = nc;
    x0 = nxo;
    y0 = nyo;
    ci = ei;
    cj = ej;
    return true;
}

// Records a removal: class counter in LDS, trench-bottom charge, hit ring.
__device__ __forceinline__ void record_hit(const PK &a, unsigned *tl, int dead, int ei, int ej,
                                           float ux, float uy)
{
    atomicAdd(&tl[dead], 1u);
    if (a.surf && dead == 4) gatomic_add(&a.surf[ej], 1ull);
    if (a.iad && dead == 4) {
        // impact angle to the plate normal (+x), 2-degree bins over [-90, 90)
        const float ang = atan2f(uy, ux);
        int bin = (int)floorf((ang + 1.57079632679f) * (float)(kIadBins / 3.14159265359));
        bin = bin < 0 ? 0 : (bin >= kIadBins ? kIadBins - 1 : bin);
        gatomic_add(&a.iad[bin], 1ull);
    }
    if (a.log.rec && ((a.log.species_mask >> a.species) & 1)) {
        unsigned long long k = atomicAdd(a.log.count, 1ull);
        long long slot = (long long)(k % (unsigned long long)a.log.capacity);
        int32_t *r = a.log.rec + 6 * slot;
        r[0] = (a.species << 8) | dead;
        r[1] = (int)(((unsigned)ei << 16) | (unsigned)ej);
        r[2] = __float_as_int(ux);
        r[3] = __float_as_int(uy);
        r[4] = (int)a.step[0];
        r[5] = 0;
    }
}

// Streaming (non-temporal) 16-byte particle loads and stores: each slot is
// read and written once per step, so they need not displace the field and
// charge arrays from the caches.
__device__ __forceinline__ nt_i4 ld_nt_i4(GLOBAL const int32_t *p)
{
    return __builtin_nontemporal_load((GLOBAL const nt_i4 *)p);
}
__device__ __forceinline__ nt_f4 ld_nt_f4(GLOBAL const float *p)
{
    return __builtin_nontemporal_load((GLOBAL const nt_f4 *)p);
}
__device__ __forceinline__ void st_nt_f4(GLOBAL float *p, float a, float b, float c, float d)
{
    nt_f4 v = {a, b, c, d};
    __builtin_nontemporal_store(v, (GLOBAL nt_f4 *)p);
}
__device__ __forceinline__ void st_nt_i4(GLOBAL int32_t *p, int a, int b, int c, int d)
{
    nt_i4 v = {a, b, c, d};
    __builtin_nontemporal_store(v, (GLOBAL nt_i4 *)p);
}

// Corner fields of the particle's cell (packed code c >= 0): from the
// block's LDS copy of the tile + 1-cell frame (origin e0i, e0j; EW x EH
// cells), or from global memory for a particle that left the frame.
__device__ __forceinline__ void cell_fields(const PK &a, const float4 *sE, int e0i, int e0j, int EW,
                                            int EH, int c, float4 &ea, float4 &eb)
{
    const Geom &g = a.g;
    const int ci = (int)((unsigned)c >> 16), cj = c & 0xFFFF;
    int li = ci - e0i, lj = cj - e0j;
    if (g.px) { if (li < 0) li += g.nx; else if (li >= g.nx) li -= g.nx; }
    if (g.py) { if (lj < 0) lj += g.ny; else if (lj >= g.ny) lj -= g.ny; }
    if (li >= 0 && li < EW && lj >= 0 && lj < EH) {
        const int m = 2 * (li * EH + lj);
        ea = sE[m];
        eb = sE[m + 1];
    } else {
        const long long cc = (long long)ci * g.ny + cj;
        ea = ld_f4(a.E4 + 2 * cc);
        eb = ld_f4(a.E4 + 2 * cc + 1);
    }
}

// Area weighting of one lane's particle (alive, in cell (ci, cj) at offsets
// (x0, y0)) into the block's LDS window of cell moments, or straight into the
// node charge when it lies outside the window.  Called by every lane of the
// wavefront (the merge of equal cells is wavefront-wide).
// Area weighting of one particle straight into the global charge (integer
// weights as in the LDS window path).
__device__ __forceinline__ void deposit_global(GLOBAL unsigned long long *rho, const Geom &g, int ci, int cj,
                                               unsigned ux, unsigned uy)
{
    const unsigned long long S = 65536ull;
    const int i1 = g.px ? wrap_hi(ci + 1, g.nx) : ci + 1;
    const int j1 = g.py ? wrap_hi(cj + 1, g.ny) : cj + 1;
    const unsigned long long X = ux, Y = uy;
    gatomic_add(&rho[(long long)ci * g.NY + cj], (S - X) * (S - Y));
    gatomic_add(&rho[(long long)i1 * g.NY + cj], X * (S - Y));
    gatomic_add(&rho[(long long)ci * g.NY + j1], (S - X) * Y);
    gatomic_add(&rho[(long long)i1 * g.NY + j1], X * Y);
}

template <int MERGE>
__device__ __forceinline__ void deposit_lane(const PK &a, unsigned long long *mA, unsigned long long *mB,
                                             int lane, bool alive, int ci, int cj, float x0, float y0,
                                             int i0, int j0, int WX, int WY, unsigned long long &nfb)
{
    const Geom &g = a.g;
    int key = -1;
    unsigned ux = 0, uy = 0;
    if (alive) {
        ux = (unsigned)floorf(x0 * 65536.0f);
        uy = (unsigned)floorf(y0 * 65536.0f);
        int wi = ci - i0, wj = cj - j0;
        if (g.px) { if (wi < 0) wi += g.nx; else if (wi >= g.nx) wi -= g.nx; }
        if (g.py) { if (wj < 0) wj += g.ny; else if (wj >= g.ny) wj -= g.ny; }
        if (wi >= 0 && wi < WX && wj >= 0 && wj < WY) {
            key = wi * WY + wj;
        } else {
            deposit_global(a.rho, g, ci, cj, ux, uy);
            nfb++;
        }
    }
    // wavefront merge of equal cells (all lanes take part)
    const unsigned m3 = ux * uy;
    if (MERGE > 0) {
        unsigned long long pend = __ballot(key >= 0);
        for (int it = 0; it < MERGE && pend; it++) {
            const int leader = __builtin_ctzll(pend);
            const int lk = __builtin_amdgcn_readlane(key, leader);
            const bool m = key == lk;
            const unsigned long long mask = __ballot(m);
            unsigned sx = m ? ux : 0u, sy = m ? uy : 0u;
            unsigned sh = m ? (m3 >> 16) : 0u, sl = m ? (m3 & 0xFFFFu) : 0u;
            wave_sum4_u32(sx, sy, sh, sl);
            if (lane == leader) {
                const unsigned long long cnt = (unsigned long long)__popcll(mask);
                const unsigned long long s3 = ((unsigned long long)sh << 16) + sl;
                atomicAdd(&mA[lk], (cnt << 45) + s3);
                atomicAdd(&mB[lk], (unsigned long long)sx | ((unsigned long long)sy << 29));
            }
            if (m) key = -1;
            pend &= ~mask;
        }
    }
    if (key >= 0) {
        atomicAdd(&mA[key], (1ull << 45) + (unsigned long long)m3);
        atomicAdd(&mB[key], (unsigned long long)ux | ((unsigned long long)uy << 29));
    }
}

// ---- block-local cell coordinates -------------------------------------------
// A particle's cell relative to the origin of the block's conductor map,
// taken into [0, n) on a periodic axis (c0w: the origin already in [0, n)
// there, nw = n; on a bounded axis c0w is the origin and nw = 0).  The field
// frame and the deposit window are fixed shifts of the same origin, so one
// wrapped coordinate serves all three LDS copies, and a step of the walk is
// one add.  An LDS copy holds the cell (origin + l) mod n at index l, so any
// representative of the cell modulo n that lands inside a copy reads the
// right entry.  Selects, not branches: the wrap costs the same on every lane.
__device__ __forceinline__ int map_rel(int c, int c0w, int nw)
{
    int l = c - c0w;
    l += l < 0 ? nw : 0;
    return l;
}

// A cell index one step from a valid one, back into [0, n) on a periodic
// axis (nw = n; nw = 0 leaves a bounded axis's index as it is).
__device__ __forceinline__ int wrap_step(int c, int n, int nw)
{
    c += c < 0 ? nw : 0;
    c -= c >= n ? nw : 0;
    return c;
}

// Whether the cell a step of the walk enters stops the particle (a conductor
// cell, or outside a bounded axis).  (lx, ly): its conductor-map coordinates;
// (gi, gj): its global ones, one cell from a valid cell, not yet wrapped.  The
// LDS map holds 1 for cells outside a bounded axis, so both tests agree.
__device__ __forceinline__ bool step_blocked(const PK &a, int lx, int ly, int gi, int gj)
{
    if ((unsigned)lx < (unsigned)a.CW && (unsigned)ly < (unsigned)a.CH)
        return a.scc[__umul24((unsigned)lx, (unsigned)a.CH) + ly] != 0;
    const Geom &g = a.g;
    if (g.px) gi = wrap_step(gi, g.nx, g.nx);
    else if (gi < 0 || gi >= g.nx) return true;
    if (g.py) gj = wrap_step(gj, g.ny, g.ny);
    else if (gj < 0 || gj >= g.ny) return true;
    return a.cell_cond[(long long)gi * g.ny + gj] != 0;
}

// push_core with the particle's cell also in conductor-map coordinates
// (lx, ly; moved with the particle).  The same arithmetic in the same order;
// a move of at most one face per axis (all but a few particles per million)
// is walked in straight-line code: for a diagonal move the earlier face first,
// compared as fx |Dy| <= fy |Dx| (ties cross x), then the other one.  Longer
// moves take the cell-by-cell walk of push_core.
__device__ __forceinline__ bool push_core_l(const PK &a, float x0, float y0, float vx0, float vy0,
                                            float4 ea, float4 eb, int ci, int cj, int &lx, int &ly,
                                            int &dead, int &ei, int &ej, float &ux, float &uy,
                                            float &nxo, float &nyo)
{
    const Geom &g = a.g;
    const float wx0 = 1.0f - x0, wy0 = 1.0f - y0;
    const float w00 = wx0 * wy0, w10 = x0 * wy0, w01 = wx0 * y0, w11 = x0 * y0;
    float ex = w00 * ea.x;
    ex = ex + w10 * ea.z;
    ex = ex + w01 * eb.x;
    ex = ex + w11 * eb.z;
    float ey = w00 * ea.y;
    ey = ey + w10 * ea.w;
    ey = ey + w01 * eb.y;
    ey = ey + w11 * eb.w;
    ux = vx0 + a.qdt * ex;
    uy = vy0 + a.qdt * ey;
    const float Dx = ux * a.dtf, Dy = uy * a.dtf;
    const float x1 = x0 + Dx, y1 = y0 + Dy;
    const float fsx = floorf(x1), fsy = floorf(y1);
    dead = -1;
    ei = ci;
    ej = cj;
    nxo = x0;
    nyo = y0;
    if (!(fabsf(fsx) < 1.0e6f && fabsf(fsy) < 1.0e6f)) {
        dead = 8;
        return false;
    }
    const int sx = (int)fsx, sy = (int)fsy;
    if (sx != 0 || sy != 0) {
        if ((unsigned)(sx + 1) <= 2u && (unsigned)(sy + 1) <= 2u) {
            const bool both = sx != 0 && sy != 0;
            bool gox = sy == 0;
            if (both) {
                const float fx = sx > 0 ? 1.0f - x0 : x0, fy = sy > 0 ? 1.0f - y0 : y0;
                gox = fx * fabsf(Dy) <= fy * fabsf(Dx);
            }
            const int d1x = gox ? sx : 0, d1y = gox ? 0 : sy;
            if (step_blocked(a, lx + d1x, ly + d1y, ci + d1x, cj + d1y)) {
                dead = gox ? (sx > 0 ? 0 : 1) : (sy > 0 ? 2 : 3);
            } else if (both && step_blocked(a, lx + sx, ly + sy, ci + sx, cj + sy)) {
                dead = gox ? (sy > 0 ? 2 : 3) : (sx > 0 ? 0 : 1);
                ei = wrap_step(ci + d1x, g.nx, a.nwx);
                ej = wrap_step(cj + d1y, g.ny, a.nwy);
            }
            if (dead >= 0) {
                const bool inbox = ei >= a.box_i_top && ej >= a.box_j_lo && ej < a.box_j_hi;
                dead += inbox ? 4 : 0;
                return false;
            }
            ei = wrap_step(ci + sx, g.nx, a.nwx);
            ej = wrap_step(cj + sy, g.ny, a.nwy);
        } else {
            walk_cells(a, x0, y0, Dx, Dy, sx, sy, dead, ei, ej);
            if (dead >= 0) return false;
        }
        lx += sx;
        ly += sy;
    }
    nxo = x1 - (float)sx;
    nyo = y1 - (float)sy;
    if (nxo >= 1.0f) nxo = 0x1.fffffep-1f;
    if (nyo >= 1.0f) nyo = 0x1.fffffep-1f;
    return true;
}

// Corner fields from conductor-map coordinates (lx, ly): the field frame's
// origin is the map's shifted by halo + 1 - kFieldFrame cells.
__device__ __forceinline__ void cell_fields_l(const PK &a, const float4 *sE, int sh, int EW, int EH, int lx,
                                              int ly, int ci, int cj, float4 &ea, float4 &eb)
{
    const int li = lx - sh, lj = ly - sh;
    if ((unsigned)li < (unsigned)EW && (unsigned)lj < (unsigned)EH) {
        const int m = 2 * (int)(__umul24((unsigned)li, (unsigned)EH) + lj);
        ea = sE[m];
        eb = sE[m + 1];
    } else {
        const long long cc = (long long)ci * a.g.ny + cj;
        ea = ld_f4(a.E4 + 2 * cc);
        eb = ld_f4(a.E4 + 2 * cc + 1);
    }
}

// deposit_lane with the deposit-window coordinates given (wi, wj: the
// conductor-map ones less 1).
template <int MERGE>
__device__ __forceinline__ void deposit_lane_l(const PK &a, unsigned long long *mA, unsigned long long *mB,
                                               int lane, bool alive, int ci, int cj, float x0, float y0,
                                               int wi, int wj, int WX, int WY, unsigned long long &nfb)
{
    int key = -1;
    unsigned ux = 0, uy = 0;
    if (alive) {
        // offsets lie in [0, 1): truncation is the floor
        ux = (unsigned)(x0 * 65536.0f);
        uy = (unsigned)(y0 * 65536.0f);
        if ((unsigned)wi < (unsigned)WX && (unsigned)wj < (unsigned)WY) {
            key = (int)__umul24((unsigned)wi, (unsigned)WY) + wj;
        } else {
            deposit_global(a.rho, a.g, ci, cj, ux, uy);
            nfb++;
        }
    }
    // both factors below 2^16: the 24-bit product is exact
    const unsigned m3 = __umul24(ux, uy);
    if (MERGE > 0) {
        unsigned long long pend = __ballot(key >= 0);
        for (int it = 0; it < MERGE && pend; it++) {
            const int leader = __builtin_ctzll(pend);
            const int lk = __builtin_amdgcn_readlane(key, leader);
            const bool m = key == lk;
            const unsigned long long mask = __ballot(m);
            unsigned sx = m ? ux : 0u, sy = m ? uy : 0u;
            unsigned sh = m ? (m3 >> 16) : 0u, sl = m ? (m3 & 0xFFFFu) : 0u;
            wave_sum4_u32(sx, sy, sh, sl);
            if (lane == leader) {
                const unsigned long long cnt = (unsigned long long)__popcll(mask);
                const unsigned long long s3 = ((unsigned long long)sh << 16) + sl;
                atomicAdd(&mA[lk], (cnt << 45) + s3);
                atomicAdd(&mB[lk], (unsigned long long)sx | ((unsigned long long)sy << 29));
            }
            if (m) key = -1;
            pend &= ~mask;
        }
    }
    if (key >= 0) {
        atomicAdd(&mA[key], (1ull << 45) + (unsigned long long)m3);
        atomicAdd(&mB[key], (unsigned long long)ux | ((unsigned long long)uy << 29));
    }
}

// One tile of particles per block (table entry): gather + push + wall test,
// then area weighting of the new positions into the block's LDS window of
// cell moments (count, sum ux, sum uy, sum ux*uy with ux, uy the 16-bit
// quantised offsets).  Lanes of a wavefront that land in the same cell are
// summed first when MERGE > 0 (up to MERGE distinct cells per wavefront),
// so runs of particles in one cell cost one LDS atomic per cell.
// Particles that drifted beyond the window add their four corner weights to
// global memory directly.  The window is flushed to the node charge at the end.
// The dispatcher hands blocks to the 8 XCDs in turn (block b to XCD b mod 8),
// each with its own L2.  In every group of 8 K blocks this gives XCD x the K
// consecutive table entries x K .. x K + K - 1 (a bijection on [0, G); a last,
// partial group is split the same way), so the blocks of one tile, which read
// the same field frame and conductor map, mostly share an L2, while every XCD
// still gets an equal share of each group.
__device__ __forceinline__ int xcd_swizzle(int b, int G)
{
    constexpr int K = 16;
    const int base = b / (8 * K) * (8 * K);
    const int n = min(8 * K, G - base);
    const int o = b - base, x = o & 7, q = n >> 3, r = n & 7;
    return base + (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + (o >> 3);
}

template <bool PUSH, int U, int MERGE>
__global__ __launch_bounds__(kPushThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_push(const PushArgs *A, Tab t)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int bid = xcd_swizzle((int)blockIdx.x, (int)gridDim.x);
    const int ku = unit_of(t, bid);
    const PushArgs &aa = A[t.id[ku]];
    const int lb = bid - t.boff[ku];
    if ((long long)lb >= aa.info[1]) return;
    const int4 ent = aa.table[lb];
    PK a = resolve(aa);
    unsigned long long *const tally = aa.tally;
    unsigned long long *const fallbacks = aa.fallbacks;
    const int tile = ent.x, start = ent.y, end = ent.z;
    const int ti = tile / a.tiles_y, tj = tile - ti * a.tiles_y;
    const int i0 = ti * a.TX - a.H, j0 = tj * a.TY - a.H;
    const int WX = a.WX, WY = a.WY, WC = WX * WY;
    // per window cell: mA = count << 45 | sum(ux*uy), mB = sum(ux) | sum(uy) << 29
    // (at most 8192 particles per block keep every field free of carries)
    unsigned long long *mA = (unsigned long long *)smem;
    unsigned long long *mB = mA + WC;
    unsigned *tl = (unsigned *)(mB + WC);
    // corner fields of the tile + 1-cell frame
    float4 *sE = (float4 *)(smem + (((size_t)WC * 16 + kNClass * 4 + 15) & ~(size_t)15));
    const int EW = a.TX + 2 * kFieldFrame, EH = a.TY + 2 * kFieldFrame;
    const int e0i = ti * a.TX - kFieldFrame, e0j = tj * a.TY - kFieldFrame;
    // conductor map of the window and a one-cell frame, after the fields
    uint8_t *scc = (uint8_t *)(sE + 2 * EW * EH);
    a.scc = scc;
    a.c0i = i0 - 1;
    a.c0j = j0 - 1;
    a.nwx = aa.g.px ? aa.g.nx : 0;
    a.nwy = aa.g.py ? aa.g.ny : 0;
    a.c0wi = a.nwx ? ((a.c0i % a.nwx) + a.nwx) % a.nwx : a.c0i;
    a.c0wj = a.nwy ? ((a.c0j % a.nwy) + a.nwy) % a.nwy : a.c0j;
    a.CW = PUSH ? WX + 2 : 0;
    a.CH = WY + 2;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const Geom g = a.g;
    for (int k = tid; k < WC; k += kPushThreads) {
        mA[k] = 0ull;
        mB[k] = 0ull;
    }
    if (tid < kNClass) tl[tid] = 0u;
    if (PUSH) {
        for (int k = tid; k < 2 * EW * EH; k += kPushThreads) {
            const int m = k >> 1, li = m / EH, lj = m - li * EH;
            int ci = e0i + li, cj = e0j + lj;
            if (g.px) ci = wrap_hi(wrap_lo(ci, g.nx), g.nx);
            if (g.py) cj = wrap_hi(wrap_lo(cj, g.ny), g.ny);
            if (ci >= 0 && ci < g.nx && cj >= 0 && cj < g.ny)
                sE[k] = ld_f4(a.E4 + 2 * ((long long)ci * g.ny + cj) + (k & 1));
        }
        for (int k = tid; k < a.CW * a.CH; k += kPushThreads) {
            const int li = k / a.CH, lj = k - li * a.CH;
            int ci = a.c0i + li, cj = a.c0j + lj;
            if (g.px) ci = ((ci % g.nx) + g.nx) % g.nx;
            if (g.py) cj = ((cj % g.ny) + g.ny) % g.ny;
            // cells outside a bounded axis are never looked up (the walk
            // tests the domain first)
            scc[k] = (ci >= 0 && ci < g.nx && cj >= 0 && cj < g.ny) ? a.cell_cond[(long long)ci * g.ny + cj] : 1;
        }
    }
    __syncthreads();

    unsigned long long nfb = 0;
    if constexpr (U == 4) {
        // 4 consecutive particles per thread per pass, moved with 16-byte
        // loads and stores where the 4 slots lie inside [start, end) (the
        // head and tail of the range go element by element).  Slots of
        // removed particles in a full vector are written back unchanged.
        // A pass's full vectors are loaded at the end of the pass before it,
        // ahead of that pass's stores: the wait at the top of a pass is then
        // for the loads alone, and their registers are not those of the
        // stores still in flight.  The wave issues them at raised priority,
        // so that they leave before other waves' arithmetic.
        nt_i4 c4 = {-1, -1, -1, -1};
        nt_f4 x4 = {0.f, 0.f, 0.f, 0.f}, y4 = x4, u4 = x4, w4 = x4;
        auto no_pass = [&]() {
            c4 = nt_i4{-1, -1, -1, -1};
            x4 = y4 = u4 = w4 = nt_f4{0.f, 0.f, 0.f, 0.f};
        };
        auto load_pass = [&](int v) {
            __builtin_amdgcn_s_setprio(3);
            c4 = ld_nt_i4(a.cell + v);
            x4 = ld_nt_f4(a.ox + v);
            y4 = ld_nt_f4(a.oy + v);
            if (PUSH) {
                u4 = ld_nt_f4(a.vx + v);
                w4 = ld_nt_f4(a.vy + v);
            }
            __builtin_amdgcn_s_setprio(0);
        };
        {
            const int v = (start & ~3) + 4 * tid;
            if (v >= start && v + 4 <= end) load_pass(v);
            else no_pass();
        }
        for (int vb = start & ~3; vb < end; vb += 4 * kPushThreads) {
            const int v = vb + 4 * tid;
            const bool full = v >= start && v + 4 <= end;
            int cv[4];
            float xv[4], yv[4], uxv[4], uyv[4];
            if (full) {
                cv[0] = c4.x; cv[1] = c4.y; cv[2] = c4.z; cv[3] = c4.w;
                xv[0] = x4.x; xv[1] = x4.y; xv[2] = x4.z; xv[3] = x4.w;
                yv[0] = y4.x; yv[1] = y4.y; yv[2] = y4.z; yv[3] = y4.w;
                uxv[0] = u4.x; uxv[1] = u4.y; uxv[2] = u4.z; uxv[3] = u4.w;
                uyv[0] = w4.x; uyv[1] = w4.y; uyv[2] = w4.z; uyv[3] = w4.w;
            } else {
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int p = v + k;
                    const bool in = p >= start && p < end;
                    cv[k] = in ? a.cell[p] : -1;
                    xv[k] = in ? a.ox[p] : 0.f;
                    yv[k] = in ? a.oy[p] : 0.f;
                    uxv[k] = (PUSH && in) ? a.vx[p] : 0.f;
                    uyv[k] = (PUSH && in) ? a.vy[p] : 0.f;
                }
            }
            bool alv[4];
            // slots holding a live particle on entry (cv[k] becomes its new code)
            unsigned live0 = 0u;
            // the field frame's origin relative to the conductor map's
            const int fsh = a.H + 1 - kFieldFrame;
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int c = cv[k];
                bool alive = false;
                int ci = 0, cj = 0, lx = -1, ly = -1;
                if (c >= 0) {
                    ci = (int)((unsigned)c >> 16);
                    cj = c & 0xFFFF;
                    lx = map_rel(ci, a.c0wi, a.nwx);
                    ly = map_rel(cj, a.c0wj, a.nwy);
                    alive = true;
                    live0 |= 1u << k;
                    if (PUSH) {
                        // the corner fields of this particle's cell only (fewer
                        // live registers than gathering all four first)
                        float4 ea, eb;
                        cell_fields_l(a, sE, fsh, EW, EH, lx, ly, ci, cj, ea, eb);
                        int dead, ei, ej;
                        float ux, uy, nxo, nyo;
                        alive = push_core_l(a, xv[k], yv[k], uxv[k], uyv[k], ea, eb, ci, cj, lx, ly,
                                            dead, ei, ej, ux, uy, nxo, nyo);
                        uxv[k] = ux;
                        uyv[k] = uy;
                        if (!alive) {
                            cv[k] = -1 - dead;
                            record_hit(a, tl, dead, ei, ej, ux, uy);
                        } else {
                            cv[k] = (int)(((unsigned)ei << 16) | (unsigned)ej);
                            xv[k] = nxo;
                            yv[k] = nyo;
                            ci = ei;
                            cj = ej;
                        }
                    }
                }
                alv[k] = alive;
                deposit_lane_l<MERGE>(a, mA, mB, lane, alive, ci, cj, xv[k], yv[k], lx - 1, ly - 1, WX, WY,
                                      nfb);
            }
            {
                // the next pass's vectors (slots v + 1024 .. v + 1027 lie at or
                // after start, so full means inside [start, end))
                const int vn = v + 4 * kPushThreads;
                if (vn + 4 <= end) load_pass(vn);
                else no_pass();
            }
            if (PUSH) {
                if (full) {
                    // every code of the vector (unchanged ones rewritten as read)
                    st_nt_i4(a.cell + v, cv[0], cv[1], cv[2], cv[3]);
                    st_nt_f4(a.vx + v, uxv[0], uxv[1], uxv[2], uxv[3]);
                    st_nt_f4(a.vy + v, uyv[0], uyv[1], uyv[2], uyv[3]);
                    st_nt_f4(a.ox + v, xv[0], xv[1], xv[2], xv[3]);
                    st_nt_f4(a.oy + v, yv[0], yv[1], yv[2], yv[3]);
                } else {
#pragma unroll
                    for (int k = 0; k < 4; k++) {
                        if (!((live0 >> k) & 1u)) continue;   // outside the range, or removed earlier
                        a.cell[v + k] = cv[k];
                        a.vx[v + k] = uxv[k];
                        a.vy[v + k] = uyv[k];
                        if (alv[k]) {
                            a.ox[v + k] = xv[k];
                            a.oy[v + k] = yv[k];
                        }
                    }
                }
            }
        }
    } else
    // U particles per thread per pass: all their loads are issued
    // before any is used, so each wave keeps several requests in flight.
    // The loop bound is uniform per block so whole wavefronts stay active.
    for (int base = start; base < end; base += U * kPushThreads) {
        int cu[U];
        float xu[U], yu[U], vxu[U], vyu[U];
        float4 eau[U], ebu[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int p = base + u * kPushThreads + tid;
            cu[u] = (p < end) ? a.cell[p] : -1;
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int p = base + u * kPushThreads + tid;
            if (p < end) {
                xu[u] = a.ox[p];
                yu[u] = a.oy[p];
                if (PUSH) {
                    vxu[u] = a.vx[p];
                    vyu[u] = a.vy[p];
                }
            }
        }
        if (PUSH) {
#pragma unroll
            for (int u = 0; u < U; u++) {
                eau[u] = ebu[u] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (cu[u] >= 0) cell_fields(a, sE, e0i, e0j, EW, EH, cu[u], eau[u], ebu[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int p = base + u * kPushThreads + tid;
            int c = cu[u];
            bool alive = false;
            float x0 = 0.f, y0 = 0.f;
            int ci = 0, cj = 0;
            if (c >= 0) {
                x0 = xu[u];
                y0 = yu[u];
                ci = (int)((unsigned)c >> 16);
                cj = c & 0xFFFF;
                alive = true;
                if (PUSH) {
                    int dead, ei, ej;
                    float vnx, vny;
                    alive = push_particle(a, p, c, x0, y0, vxu[u], vyu[u], eau[u], ebu[u], ci, cj,
                                          dead, ei, ej, vnx, vny);
                    if (!alive) record_hit(a, tl, dead, ei, ej, vnx, vny);
                }
            }
            deposit_lane<MERGE>(a, mA, mB, lane, alive, ci, cj, x0, y0, i0, j0, WX, WY, nfb);
        }
    }
    if (nfb) atomicAdd(fallbacks, nfb);
    __syncthreads();
    // flush: node (wa, wb) of the window collects the four cells around it
    const unsigned long long S = 65536ull;
    const int WN = (WX + 1) * (WY + 1);
    for (int k = tid; k < WN; k += kPushThreads) {
        const int wa = k / (WY + 1), wb = k - wa * (WY + 1);
        unsigned long long v = 0ull;
        bool any = false;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int ca = wa - (q & 1), cb = wb - (q >> 1);
            if (ca < 0 || ca >= WX || cb < 0 || cb >= WY) continue;
            const int m = ca * WY + cb;
            const unsigned long long A = mA[m];
            if (A == 0ull) continue;
            any = true;
            const unsigned long long B = mB[m];
            const unsigned long long M0 = A >> 45, M3 = A & ((1ull << 45) - 1ull);
            const unsigned long long M1 = B & ((1ull << 29) - 1ull), M2 = B >> 29;
            if (q == 0) v += S * S * M0 - S * M1 - S * M2 + M3;  // node is the cell's 00 corner
            else if (q == 1) v += S * M1 - M3;                    // 10 corner of cell (wa-1, wb)
            else if (q == 2) v += S * M2 - M3;                    // 01 corner of cell (wa, wb-1)
            else v += M3;                                         // 11 corner of cell (wa-1, wb-1)
        }
        if (!any || v == 0ull) continue;
        int gi = i0 + wa, gj = j0 + wb;
        if (g.px) { gi = ((gi % g.NX) + g.NX) % g.NX; }
        else if (gi < 0 || gi >= g.NX) continue;
        if (g.py) { gj = ((gj % g.NY) + g.NY) % g.NY; }
        else if (gj < 0 || gj >= g.NY) continue;
        gatomic_add(&a.rho[(long long)gi * g.NY + gj], v);
    }
    if (PUSH && tid < kNClass && tl[tid]) atomicAdd(&tally[tid], (unsigned long long)tl[tid]);
}

template <bool PUSH>
static void launch_push_t(const PushArgs *A, const Tab &t, int unroll, int merge, size_t lds,
                          hipStream_t s)
{
    const dim3 gr(tab_blocks(t)), bl(kPushThreads);
#define PUSH_CASE(U, M)                                                                   \
    if (unroll == U && merge == M) {                                                      \
        hipLaunchKernelGGL((k_push<PUSH, U, M>), gr, bl, lds, s, A, t);                   \
        return;                                                                           \
    }
    PUSH_CASE(1, 0) PUSH_CASE(2, 0) PUSH_CASE(4, 0)
    PUSH_CASE(1, 2) PUSH_CASE(2, 2) PUSH_CASE(4, 2)
    PUSH_CASE(1, 4) PUSH_CASE(2, 4) PUSH_CASE(4, 4)
#undef PUSH_CASE
    hipLaunchKernelGGL((k_push<PUSH, 2, 0>), gr, bl, lds, s, A, t);
}

void launch_push(const PushArgs *A, const Tab &t, bool push, int unroll, int merge, size_t lds,
                 hipStream_t s)
{
    if (!t.n) return;
    if (push) launch_push_t<true>(A, t, unroll, merge, lds, s);
    else launch_push_t<false>(A, t, unroll, merge, lds, s);
}

// Leapfrog start: v -= (alpha dt / 2) E(x), same gather as the push.
__global__ void k_rewind(const PushArgs *A, Tab t)
{
    const int ku = unit_of(t, (int)blockIdx.x);
    const PushArgs &aa = A[t.id[ku]];
    const long long p = (long long)((int)blockIdx.x - t.boff[ku]) * blockDim.x + threadIdx.x;
    if (p >= aa.info[2 + aa.info[7]]) return;
    const PK a = resolve(aa);
    const int c = a.cell[p];
    if (c < 0) return;
    const int ci = (int)((unsigned)c >> 16), cj = c & 0xFFFF;
    const long long cc = (long long)ci * a.g.ny + cj;
    const float4 ea = ld_f4(a.E4 + 2 * cc), eb = ld_f4(a.E4 + 2 * cc + 1);
    const float x0 = a.ox[p], y0 = a.oy[p];
    const float wx0 = 1.0f - x0, wy0 = 1.0f - y0;
    const float w00 = wx0 * wy0, w10 = x0 * wy0, w01 = wx0 * y0, w11 = x0 * y0;
    float ex = w00 * ea.x;
    ex = ex + w10 * ea.z;
    ex = ex + w01 * eb.x;
    ex = ex + w11 * eb.z;
    float ey = w00 * ea.y;
    ey = ey + w10 * ea.w;
    ey = ey + w01 * eb.y;
    ey = ey + w11 * eb.w;
    a.vx[p] = a.vx[p] - a.hq * ex;
    a.vy[p] = a.vy[p] - a.hq * ey;
}

void launch_rewind(const PushArgs *A, const Tab &t, hipStream_t s)
{
    if (t.n) hipLaunchKernelGGL(k_rewind, dim3(tab_blocks(t)), dim3(256), 0, s, A, t);
}

// ---------------------------------------------------------------------------
// diagnostics (not on the stepping path): float64 sums in a fixed order
// ---------------------------------------------------------------------------

__device__ __forceinline__ void diag_block_sum(double v, double *part)
{
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Ion recycling after a push: every slot whose ion that push removed at a
// wall or conductor (code -1 - class, class 0..7) takes a thermal ion in the
// bulk rows, and the new ion's charge goes straight into rho.  The push
// leaves the lost ion's kicked v_x and its offsets before the move in the
// slot; with the step they form the generator's counter.  One thread per
// slot of the storage set in use.
__global__ __launch_bounds__(256) void k_recycle(const PushArgs *A, Tab t)
{
    const int ku = unit_of(t, (int)blockIdx.x);
    const PushArgs &a = A[t.id[ku]];
    const int set = (int)a.info[7];
    const long long p = (long long)((int)blockIdx.x - t.boff[ku]) * 256 + threadIdx.x;
    if (p >= a.info[2 + set]) return;
    GLOBAL int32_t *cell = to_global(a.cell[set]);
    const int c = cell[p];
    if (c >= 0 || c < -8) return;
    GLOBAL float *ox = to_global(a.ox[set]), *oy = to_global(a.oy[set]);
    GLOBAL float *vx = to_global(a.vx[set]), *vy = to_global(a.vy[set]);
    const NewIon n = recycled_ion((unsigned long long)*a.step, vx[p], ox[p], oy[p], a.recycle_key[0],
                                  a.recycle_key[1], a.recycle_rows, a.g.ny, a.recycle_vth);
    cell[p] = (int)(((unsigned)n.ci << 16) | (unsigned)n.cj);
    ox[p] = n.ox;
    oy[p] = n.oy;
    vx[p] = n.vx;
    vy[p] = n.vy;
    deposit_global(to_global(a.rho), a.g, n.ci, n.cj, (unsigned)floorf(n.ox * 65536.0f),
                   (unsigned)floorf(n.oy * 65536.0f));
}

void launch_recycle(const PushArgs *A, const Tab &t, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_recycle, dim3(tab_blocks(t)), dim3(256), 0, s, A, t);
}

__global__ __launch_bounds__(256) void k_kinetic(const PushArgs *A, int unit, double *part)
{
    const PushArgs &aa = A[unit];
    const int set = (int)aa.info[7];
    const long long n = aa.info[2 + set];
    const int32_t *cell = aa.cell[set];
    const float *vx = aa.vx[set], *vy = aa.vy[set];
    double s = 0.0;
    for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += (long long)gridDim.x * 256)
        if (cell[p] >= 0) s += (double)vx[p] * vx[p] + (double)vy[p] * vy[p];
    diag_block_sum(s, part);
}

__global__ __launch_bounds__(256) void k_field_energy(const Inst *insts, int inst, double *part)
{
    const Inst &I = insts[inst];
    const Geom g = I.g;
    const long long n = (long long)g.NX * g.NY;
    double s = 0.0;
    for (long long k = (long long)blockIdx.x * 256 + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
        const int i = (int)(k / g.NY), j = (int)(k % g.NY);
        const float2 e = node_field(g, I.node_cond, I.phi, i, j);
        s += (double)e.x * e.x + (double)e.y * e.y;
    }
    diag_block_sum(0.5 * s, part);
}

__global__ void k_sum_partials(const double *part, int n, double *out)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < n; k++) s += part[k];
    *out = s;
}

void launch_kinetic(const PushArgs *A, int unit, double *part, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_kinetic, dim3(kDiagBlocks), dim3(256), 0, s, A, unit, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, kDiagBlocks, out);
}

void launch_field_energy(const Inst *I, int inst, double *part, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_field_energy, dim3(kDiagBlocks), dim3(256), 0, s, I, inst, part);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, part, kDiagBlocks, out);
}

// ---------------------------------------------------------------------------
// re-binning: counting sort of live particles by tile (order inside a tile
// is arbitrary; results never depend on particle order)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int tile_of(int c, int lx, int ly, int tiles_y)
{
    const int i = (int)((unsigned)c >> 16), j = c & 0xFFFF;
    return (i >> lx) * tiles_y + (j >> ly);
}

// Adds 1 per active lane to counters[key], one atomic per distinct key in
// the wavefront; returns the lane's slot (previous value + rank).
__device__ __forceinline__ unsigned wave_add(unsigned *counters, int key, bool active)
{
    unsigned mine = 0;
    const int lane = __lane_id();
    unsigned long long pend = __ballot(active);
    while (pend) {
        const int leader = __builtin_ctzll(pend);
        const int lk = __shfl(key, leader, 64);
        const unsigned long long m = __ballot(active && key == lk) & pend;
        unsigned base = 0;
        if (lane == leader) base = atomicAdd(&counters[lk], (unsigned)__popcll(m));
        base = __shfl(base, leader, 64);
        if ((m >> lane) & 1ull) mine = base + (unsigned)__popcll(m & ((1ull << lane) - 1ull));
        pend &= ~m;
    }
    return mine;
}

// A slot is binned when its code is non-negative and names a cell of the
// grid; a non-negative code outside the grid is counted in bad[0] and dropped.
__device__ __forceinline__ bool live_code(int c, int nx, int ny)
{
    return c >= 0 && (int)((unsigned)c >> 16) < nx && (c & 0xFFFF) < ny;
}

// Count and scatter work in blocks of kBinPer consecutive slots.  Between
// re-binnings particles drift less than a tile, so a block's particles lie
// in a 5 x 5 box of tiles centred on its home tile (the tile of the first
// live particle among thread 0's slots, which may itself have moved a tile;
// tile indices taken modulo the tile grid, so the box is an index map
// whatever the boundaries).  The scatter counts its particles per box tile
// in LDS (one LDS atomic per distinct tile per wavefront), reserves that
// many consecutive destination slots with one global atomic per tile and
// hands them out in LDS; particles outside the box use global
// wavefront-aggregated atomics.
constexpr int kBinPer = 2048;
constexpr int kBox = 5;
constexpr int kBoxN = kBox * kBox;

// Source (info[7]) and destination sets of a re-binning.
struct BView {
    const int32_t *cell;
    const float *ox, *oy, *vx, *vy;
    int32_t *cell2;
    float *ox2, *oy2, *vx2, *vy2;
    long long slots;
    int src, dst;
};

__device__ __forceinline__ BView bview(const BinArgs &a)
{
    BView v;
    v.src = (int)a.info[7];
    v.dst = 1 - v.src;
    v.cell = a.cell[v.src];
    v.ox = a.ox[v.src];
    v.oy = a.oy[v.src];
    v.vx = a.vx[v.src];
    v.vy = a.vy[v.src];
    v.cell2 = a.cell[v.dst];
    v.ox2 = a.ox[v.dst];
    v.oy2 = a.oy[v.dst];
    v.vx2 = a.vx[v.dst];
    v.vy2 = a.vy[v.dst];
    v.slots = a.info[2 + v.src];
    return v;
}

// A block's box: tile rows ti .. ti+kBox-1 and columns tj .. tj+kBox-1 (modulo tx, ty).
struct TileBox {
    int ti, tj, tx, ty;
    bool on;
};

// Local index of the tile of live code c in the box, or -1.
__device__ __forceinline__ int box_index(const TileBox &b, int c, int lx, int ly)
{
    if (!b.on) return -1;
    int di = (int)(((unsigned)c >> 16) >> lx) - b.ti, dj = (int)((unsigned)(c & 0xFFFF) >> ly) - b.tj;
    if (di < 0) di += b.tx;
    else if (di >= b.tx) di -= b.tx;
    if (dj < 0) dj += b.ty;
    else if (dj >= b.ty) dj -= b.ty;
    return (di < kBox && dj < kBox) ? di * kBox + dj : -1;
}

// Global tile of local index k of the box.
__device__ __forceinline__ int box_tile(const TileBox &b, int k)
{
    int ti = b.ti + k / kBox, tj = b.tj + k % kBox;
    if (ti < 0) ti += b.tx;
    else if (ti >= b.tx) ti -= b.tx;
    if (tj < 0) tj += b.ty;
    else if (tj >= b.ty) tj -= b.ty;
    return ti * b.ty + tj;
}

// Scatter pass: loads the block's cell codes (all loads issued before
// use), sets up its box (shared home) and counts the live ones per box tile
// in hist (zeroed here).
constexpr int kBinRP = kBinPer / 256;
__device__ __forceinline__ TileBox bin_local_count(const BinArgs &a, const BView &v, long long lo, long long hi,
                                                   unsigned *hist, int *home, int (&cv)[kBinRP])
{
#pragma unroll
    for (int r8 = 0; r8 < kBinRP; r8++) {
        const long long p = lo + r8 * 256 + threadIdx.x;
        cv[r8] = p < hi ? v.cell[p] : -1;
    }
    if (threadIdx.x < kBoxN) hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) {
        int h = -1;
#pragma unroll
        for (int r8 = 0; r8 < kBinRP; r8++)
            if (h < 0 && live_code(cv[r8], a.nx, a.ny)) h = cv[r8];
        *home = h;
    }
    __syncthreads();
    TileBox b;
    const int h = *home;
    b.on = h >= 0;
    b.ty = a.tiles_y;
    b.tx = a.ntiles / a.tiles_y;
    b.ti = b.on ? (int)(((unsigned)h >> 16) >> a.lx) - kBox / 2 : 0;
    b.tj = b.on ? (int)((unsigned)(h & 0xFFFF) >> a.ly) - kBox / 2 : 0;
#pragma unroll
    for (int r8 = 0; r8 < kBinRP; r8++) {
        const int c = cv[r8];
        const bool act = live_code(c, a.nx, a.ny);
        const int k = act ? box_index(b, c, a.lx, a.ly) : -1;
        wave_add(hist, k < 0 ? 0 : k, act && k >= 0);
    }
    __syncthreads();
    return b;
}

// Count pass: the block's live particles per tile in an LDS histogram over
// the whole tile grid (tiles beyond kCountLds in global counts), added to
// the global counts once per non-zero tile; codes outside the grid in bad.
// (No box here: the count has no home tile to wait for, and the scatter
// places every particle counted for a tile in that tile's range whichever
// path counted it.)
constexpr int kCountLds = 2048;

__global__ __launch_bounds__(256) void k_bin_count(const BinArgs *B, Tab t)
{
    __shared__ unsigned hist[kCountLds];
    const int ku = unit_of(t, (int)blockIdx.x);
    const BinArgs &a = B[t.id[ku]];
    const BView v = bview(a);
    const long long n = v.slots;
    const long long lo = (long long)((int)blockIdx.x - t.boff[ku]) * kBinPer;
    if (lo >= n) return;
    const long long hi = lo + kBinPer < n ? lo + kBinPer : n;
    const int nl = a.ntiles < kCountLds ? a.ntiles : kCountLds;
    int cv[kBinRP];
#pragma unroll
    for (int r8 = 0; r8 < kBinRP; r8++) {
        const long long p = lo + r8 * 256 + threadIdx.x;
        cv[r8] = p < hi ? v.cell[p] : -1;
    }
    for (int k = threadIdx.x; k < nl; k += 256) hist[k] = 0u;
    __syncthreads();
#pragma unroll
    for (int r8 = 0; r8 < kBinRP; r8++) {
        const int c = cv[r8];
        const bool act = live_code(c, a.nx, a.ny);
        if (c >= 0 && !act) atomicAdd(a.bad, 1ull);
        const int key = act ? tile_of(c, a.lx, a.ly, a.tiles_y) : 0;
        wave_add(hist, key, act && key < kCountLds);
        wave_add(a.counts, key, act && key >= kCountLds);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nl; k += 256)
        if (hist[k]) atomicAdd(&a.counts[k], hist[k]);
}

// Single work-group: exclusive scans of the tile counts and of the blocks
// per tile; writes the cursor for the scatter and the totals.
__global__ __launch_bounds__(1024) void k_bin_scan(const BinArgs *B, Tab t)
{
    const BinArgs &a = B[t.id[blockIdx.x]];
    __shared__ unsigned long long sp[1024], sb[1024];
    const int tid = threadIdx.x, nt = blockDim.x;
    const int per = (a.ntiles + nt - 1) / nt;
    const int lo = tid * per, hi = min(a.ntiles, lo + per);
    unsigned long long s = 0, sbk = 0;
    for (int t = lo; t < hi; t++) {
        unsigned c = a.counts[t];
        s += c;
        sbk += (c + a.chunk - 1) / a.chunk;
    }
    sp[tid] = s;
    sb[tid] = sbk;
    __syncthreads();
    for (int o = 1; o < nt; o <<= 1) {
        unsigned long long x = tid >= o ? sp[tid - o] : 0, y = tid >= o ? sb[tid - o] : 0;
        __syncthreads();
        sp[tid] += x;
        sb[tid] += y;
        __syncthreads();
    }
    unsigned long long off = sp[tid] - s, boff = sb[tid] - sbk;
    for (int t = lo; t < hi; t++) {
        unsigned c = a.counts[t];
        a.offsets[t] = (unsigned)off;
        a.cursor[t] = (unsigned)off;
        a.boff[t] = (unsigned)boff;
        off += c;
        boff += (c + a.chunk - 1) / a.chunk;
    }
    if (tid == nt - 1) {
        a.info[0] = (long long)sp[tid];
        a.info[1] = (long long)sb[tid];
        a.info[2 + (1 - (int)a.info[7])] = (long long)sp[tid];
        // the binned slots and their push blocks: particles appended later
        // (secondary emission) get push blocks after these
        a.info[4] = (long long)sp[tid];
        a.info[5] = (long long)sb[tid];
    }
}

// Push-block table of the new set; clears the tile counts for the next
// re-binning.
__global__ void k_bin_table(const BinArgs *B, Tab tb)
{
    const int ku = unit_of(tb, (int)blockIdx.x);
    const BinArgs &a = B[tb.id[ku]];
    const int t = ((int)blockIdx.x - tb.boff[ku]) * blockDim.x + threadIdx.x;
    if (t >= a.ntiles) return;
    const unsigned c = a.counts[t], o = a.offsets[t], b0 = a.boff[t];
    const unsigned nb = (c + a.chunk - 1) / a.chunk;
    for (unsigned k = 0; k < nb; k++) {
        unsigned s = o + k * a.chunk;
        unsigned e = min(o + c, s + (unsigned)a.chunk);
        a.table[b0 + k] = make_int4(t, (int)s, (int)e, 0);
    }
    a.counts[t] = 0u;
}

__device__ __forceinline__ unsigned gcd_u(unsigned x, unsigned y)
{
    while (y) {
        unsigned t = x % y;
        x = y;
        y = t;
    }
    return x;
}

// Scatter: the m particles a block sends to tile t take its reserved slots
// base..base+m-1, in the order r -> (r * stride) mod m (r = arrival rank,
// stride near 0.618 m and coprime to m), so runs of particles from one cell
// are spread over the tile's range (the lanes of a wavefront in the push then
// mostly deposit into different cells).  Each of the five arrays passes
// through LDS: coalesced loads of the block's slots, stores into LDS at the
// staging position, then coalesced stores of the staged runs to their
// consecutive destination slots.
// One array of the block through LDS: values (in registers, slot order) to
// their staging positions, then the staged runs to their destination slots.
// Staged moves of two arrays at a time (the cell codes travel as float
// bits): each thread puts its particles' values at their staging positions,
// then consecutive threads write consecutive destinations (the tile ranges
// are contiguous).  c0: the first array holds cell codes.  d1 null: one array.
__device__ __forceinline__ void bin_move2(const float (&v0)[kBinRP], float *d0, int32_t *c0, const float (&v1)[kBinRP],
                                          float *d1, const int (&qv)[kBinRP], const unsigned *dst, float *buf0,
                                          float *buf1, unsigned total)
{
#pragma unroll
    for (int r8 = 0; r8 < kBinRP; r8++)
        if (qv[r8] >= 0) {
            buf0[qv[r8]] = v0[r8];
            if (d1) buf1[qv[r8]] = v1[r8];
        }
    __syncthreads();
    for (unsigned q = threadIdx.x; q < total; q += 256) {
        const unsigned d = dst[q];
        if (c0) c0[d] = __float_as_int(buf0[q]);
        else d0[d] = buf0[q];
        if (d1) d1[d] = buf1[q];
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_bin_scatter(const BinArgs *B, Tab tb)
{
    constexpr int RP = kBinPer / 256;
    __shared__ float buf0[kBinPer], buf1[kBinPer];       // staging of two arrays
    __shared__ unsigned dst[kBinPer];                    // destination slot per staging position
    __shared__ unsigned hist[kBoxN], base[kBoxN], loff[kBoxN], mstr[kBoxN];
    __shared__ unsigned total;
    __shared__ int home;
    const int ku = unit_of(tb, (int)blockIdx.x);
    const BinArgs &a = B[tb.id[ku]];
    const BView v = bview(a);
    const long long n = v.slots;
    const long long lo = (long long)((int)blockIdx.x - tb.boff[ku]) * kBinPer;
    if (lo >= n) return;
    const long long hi = lo + kBinPer < n ? lo + kBinPer : n;
    // every load of the block's slots issued up front
    float fv[4][RP];
    const float *fsrc[4] = {v.ox, v.oy, v.vx, v.vy};
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
        for (int r8 = 0; r8 < RP; r8++) {
            const long long p = lo + r8 * 256 + threadIdx.x;
            fv[f][r8] = p < hi ? fsrc[f][p] : 0.0f;
        }
    int cv[RP];
    const TileBox bx = bin_local_count(a, v, lo, hi, hist, &home, cv);
    // per box tile: a destination range, the staging offset, and a stride
    // coprime to the count that spreads runs of particles from one cell over
    // the tile's range (runs would serialise a wavefront's LDS atomics in the
    // push)
    if (threadIdx.x < kBoxN) {
        const int k = threadIdx.x;
        const unsigned m = hist[k];
        if (m) {
            base[k] = atomicAdd(&a.cursor[box_tile(bx, k)], m);
            unsigned st = (unsigned)(0.618034f * (float)m) | 1u;
            while (gcd_u(st, m) != 1u) st++;
            mstr[k] = (m << 16) | (st % m);
        }
    }
    if (threadIdx.x == 0) {
        unsigned off = 0;
        for (int k = 0; k < kBoxN; k++) {
            loff[k] = off;
            off += hist[k];
        }
        total = off;
    }
    __syncthreads();
    if (threadIdx.x < kBoxN) hist[threadIdx.x] = 0u;     // the rank counters of the pass below
    __syncthreads();
    int qv[RP];                                           // staging position of each own slot, or -1
#pragma unroll
    for (int r8 = 0; r8 < RP; r8++) {
        const int c = cv[r8];
        const bool act = live_code(c, a.nx, a.ny);
        const int k = act ? box_index(bx, c, a.lx, a.ly) : -1;
        const bool loc = act && k >= 0;
        const unsigned r = wave_add(hist, loc ? k : 0, loc);
        const unsigned d1 = wave_add(a.cursor, act ? tile_of(c, a.lx, a.ly, a.tiles_y) : 0, act && !loc);
        int qp = -1;
        if (loc) {
            const unsigned ms = mstr[k];
            const unsigned q = loff[k] + (r * (ms & 0xFFFFu)) % (ms >> 16);
            qp = (int)q;
            dst[q] = base[k] + (q - loff[k]);
        } else if (act) {
            v.cell2[d1] = c;
            v.ox2[d1] = fv[0][r8];
            v.oy2[d1] = fv[1][r8];
            v.vx2[d1] = fv[2][r8];
            v.vy2[d1] = fv[3][r8];
        }
        qv[r8] = qp;
    }
    __syncthreads();
    const unsigned nq = total;
    float cf[RP];
#pragma unroll
    for (int r8 = 0; r8 < RP; r8++) cf[r8] = __int_as_float(cv[r8]);
    bin_move2(cf, nullptr, v.cell2, fv[0], v.ox2, qv, dst, buf0, buf1, nq);
    bin_move2(fv[1], v.oy2, nullptr, fv[2], v.vx2, qv, dst, buf0, buf1, nq);
    bin_move2(fv[3], v.vy2, nullptr, fv[3], nullptr, qv, dst, buf0, buf1, nq);
}

// The destination set becomes the set in use.
__global__ void k_bin_flip(const BinArgs *B, Tab t)
{
    const BinArgs &a = B[t.id[blockIdx.x]];
    a.info[7] = 1 - a.info[7];
}

// Tabs: tcount/tscatter cover ceil(slots / kBinPer) blocks per unit, tscan
// one block per unit, ttable ceil(ntiles / 256) blocks per unit.
void launch_bin(const BinArgs *B, const Tab &tcount, const Tab &tscan, const Tab &ttable,
                hipStream_t s)
{
    if (!tscan.n) return;
    if (tab_blocks(tcount)) hipLaunchKernelGGL(k_bin_count, dim3(tab_blocks(tcount)), dim3(256), 0, s, B, tcount);
    hipLaunchKernelGGL(k_bin_scan, dim3(tscan.n), dim3(1024), 0, s, B, tscan);
    hipLaunchKernelGGL(k_bin_table, dim3(tab_blocks(ttable)), dim3(256), 0, s, B, ttable);
    if (tab_blocks(tcount)) hipLaunchKernelGGL(k_bin_scatter, dim3(tab_blocks(tcount)), dim3(256), 0, s, B, tcount);
    hipLaunchKernelGGL(k_bin_flip, dim3(tscan.n), dim3(1), 0, s, B, tscan);
}

int bin_per_block() { return kBinPer; }

// Sum of a node charge array (exact integer sum).
__global__ void k_rho_sum(const unsigned long long *rho, long long n, unsigned long long *out)
{
    __shared__ unsigned long long sh[4];
    long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long st = (long long)gridDim.x * blockDim.x;
    unsigned long long s = 0;
    for (; k < n; k += st) s += rho[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, sh[0] + sh[1] + sh[2] + sh[3]);
}

void launch_rho_sum(const unsigned long long *rho, long long n, unsigned long long *out,
                    hipStream_t s)
{
    long long nb = (n + 255) / 256;
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_rho_sum, dim3((unsigned)nb), dim3(256), 0, s, rho, n, out);
}

// ---------------------------------------------------------------------------
// secondary electron emission at the trench surfaces (Sec. IV; constant
// yield per impact, see pic_config.see_yield)
// ---------------------------------------------------------------------------

// The removals logged since the last call (grid-stride over the ring):
// every trench-surface removal (classes 4, 6, 7) of a species with a yield
// draws from Philox4x32-10, counter (step, packed cell, bits of the kicked
// velocity), key (k0, k1), and with (r0 >> 8) < thresh frees an electron:
// on the struck face of the cell (normal offset the largest float below 1
// on the cell's high side, 0 on its low side; along it (r1 >> 8) 2^-24),
// normal speed vth sqrt(-2 ln u) away from the wall and tangential velocity
// vth sqrt(-2 ln u') cos(2 pi u'') from the draw with key (k0, k1 + 1)
// (u = ((q0 >> 8) + 1) 2^-24, u' = ((q1 >> 8) + 1) 2^-24, u'' = (q2 >> 8)
// 2^-24, in double, rounded to float).  Each takes a slot after species 0's
// slots (a counter; beyond the capacity it is dropped and counted) and adds
// its charge to rho.  Records overwritten before this call are counted as
// dropped.
__global__ __launch_bounds__(256) void k_emit(const SeeArgs *A, Tab t)
{
    const int ku = unit_of(t, (int)blockIdx.x);
    const SeeArgs &a = A[t.id[ku]];
    const int lb = (int)blockIdx.x - t.boff[ku];
    const unsigned long long total = *a.log_count, done = a.misc[0];
    const unsigned long long cap = (unsigned long long)a.log_capacity;
    const unsigned long long first = total - done > cap ? total - cap : done;
    if (lb == 0 && threadIdx.x == 0 && first > done) atomicAdd(&a.misc[3], first - done);
    const int set = (int)a.info[7];
    const long long slots0 = a.info[2 + set];
    GLOBAL int32_t *cell = to_global(a.cell[set]);
    GLOBAL float *ox = to_global(a.ox[set]), *oy = to_global(a.oy[set]);
    GLOBAL float *vx = to_global(a.vx[set]), *vy = to_global(a.vy[set]);
    const float below1 = 0x1.fffffep-1f;
    for (unsigned long long k = first + (unsigned long long)lb * 256 + threadIdx.x; k < total;
         k += (unsigned long long)kEmitBlocks * 256) {
        const int32_t *r = a.rec + 6 * (long long)(k % cap);
        const int sc = r[0], cls = sc & 0xFF, sp = sc >> 8;
        if ((cls != 4 && cls != 6 && cls != 7) || sp < 0 || sp > 1 || a.thresh[sp] == 0u) continue;
        const unsigned c0 = (unsigned)r[4], c1 = (unsigned)r[1], c2 = (unsigned)r[2], c3 = (unsigned)r[3];
        const Philox4 d = philox4x32_10(c0, c1, c2, c3, a.key[0], a.key[1]);
        if ((d.x >> 8) >= a.thresh[sp]) continue;
        const Philox4 q = philox4x32_10(c0, c1, c2, c3, a.key[0], a.key[1] + 1u);
        const float along = (float)(d.y >> 8) * 0x1p-24f;
        const double u1 = (double)((q.x >> 8) + 1u) * 0x1p-24, u2 = (double)((q.y >> 8) + 1u) * 0x1p-24;
        const double u3 = (double)(q.z >> 8) * 0x1p-24;
        const double vn = a.vth * sqrt(-2.0 * log(u1));
        const double vt = a.vth * sqrt(-2.0 * log(u2)) * cos(6.283185307179586 * u3);
        float nox, noy, nvx, nvy;
        if (cls == 4) {             // +x face (the bottom): back along -x
            nox = below1; noy = along; nvx = (float)(-vn); nvy = (float)vt;
        } else if (cls == 6) {      // +y face: back along -y
            nox = along; noy = below1; nvx = (float)vt; nvy = (float)(-vn);
        } else {                    // -y face: back along +y
            nox = along; noy = 0.0f; nvx = (float)vt; nvy = (float)vn;
        }
        const long long slot = slots0 + (long long)atomicAdd(&a.misc[1], 1ull);
        if (slot >= a.capacity) {
            atomicAdd(&a.misc[3], 1ull);
            continue;
        }
        cell[slot] = r[1];
        ox[slot] = nox;
        oy[slot] = noy;
        vx[slot] = nvx;
        vy[slot] = nvy;
        const int ci = (int)((unsigned)r[1] >> 16), cj = r[1] & 0xFFFF;
        deposit_global(to_global(a.rho), a.g, ci, cj, (unsigned)floorf(nox * 65536.0f),
                       (unsigned)floorf(noy * 65536.0f));
    }
}

// After k_emit: the slots of species 0 grow by the electrons that found
// room, the push table gets blocks of `chunk` slots over everything past the
// binned slots (on tile 0's window; the push reads other cells' fields and
// deposits their charge through its global paths), and the ring position
// and counters move on.
__global__ void k_emit_finish(const SeeArgs *A, Tab t)
{
    const SeeArgs &a = A[t.id[unit_of(t, (int)blockIdx.x)]];
    const int set = (int)a.info[7];
    const long long slots0 = a.info[2 + set];
    const long long want = (long long)a.misc[1];
    const long long room = a.capacity > slots0 ? a.capacity - slots0 : 0;
    const long long got = want < room ? want : room;
    const long long slots = slots0 + got;
    const long long t0 = a.info[4], nb0 = a.info[5];
    const long long nb = slots > t0 ? (slots - t0 + a.chunk - 1) / a.chunk : 0;
    for (long long k = threadIdx.x; k < nb; k += blockDim.x) {
        const long long s0 = t0 + k * a.chunk;
        const long long s1 = s0 + a.chunk < slots ? s0 + a.chunk : slots;
        a.table[nb0 + k] = make_int4(0, (int)s0, (int)s1, 0);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.info[2 + set] = slots;
        a.info[1] = nb0 + nb;
        a.misc[0] = *a.log_count;
        a.misc[1] = 0ull;
        a.misc[2] += (unsigned long long)got;
    }
}

void launch_emit(const SeeArgs *A, const Tab &t, const Tab &t1, hipStream_t s)
{
    if (!t.n) return;
    hipLaunchKernelGGL(k_emit, dim3(tab_blocks(t)), dim3(256), 0, s, A, t);
    hipLaunchKernelGGL(k_emit_finish, dim3(tab_blocks(t1)), dim3(64), 0, s, A, t1);
}

} // namespace pic
