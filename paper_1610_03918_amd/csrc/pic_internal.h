// Internal interface between the gfx950 kernels (pic_kernels.hip) and the
// host runtime behind the C ABI (pic_runtime.cpp).  Not installed.
//
// Every kernel works on a batch of independent instances (one for pic_init,
// up to kMaxInst for pic_batch_init).  Per-instance state lives in a device
// array of Inst descriptors; a launch covers the blocks of several units
// (instances, or instance x species pairs) listed in a Tab passed by value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kMaxLev = 16;
constexpr int kNClass = 9;
constexpr int kIadBins = 90;     // 2-degree bins of the bottom-impact angle, -90 .. 90 degrees
constexpr int kDiagBlocks = 512; // blocks (and partial sums) of the diagnostic reductions
constexpr int kMaxInst = 16;
constexpr int kMaxUnits = 2 * kMaxInst;
constexpr int kGridBX = 64;      // grid kernels: 64 x 4 threads over (y, x) nodes
constexpr int kGridBY = 4;
constexpr int kPushThreads = 256;
constexpr int kFieldFrame = 1;    // cells around a push tile whose corner fields the block stages in LDS

struct Geom {
    int nx, ny;     // cells
    int NX, NY;     // nodes
    int px, py;     // periodic axes
};

// Slots of the float64 scalar block and the int flag block of an instance.
enum {
    S_BB = 0,    // ||b||^2 over unknowns
    S_RR64,      // ||b - A phi||^2 (float64 residual)
    S_RZ,        // r.z of the current inner iteration
    S_RZOLD,
    S_PQ,        // p.Ap
    S_RR,        // inner ||r||^2
    S_RR0,       // inner ||r0||^2
    S_ETA2,      // inner stop ratio (squared)
    S_SUM,       // scratch sum (mean projection)
    S_PIN,       // value of the pinned node (fully periodic gauge)
    S_RELRES,    // last float64 relative residual
    S_RELRES0,   // relative residual at the start of the solve
    S_CG_ALPHA,  // step length of the next CG step (multigrid-preconditioned form)
    S_CG_BETA,   // direction coefficient of the next CG step
    S_CG_GAMMA,  // r.z of the last V-cycle
    S_WORST,     // largest relative residual of a potential that was pushed with unconverged
    S_CG_NALPHA, // alpha, beta and r.z of the step in progress (multigrid form): written by
    S_CG_NBETA,  //   the level-0 down kernel that computes them, moved to S_CG_* by the
    S_CG_NGAMMA, //   step's update (the kernel's other blocks still read the old ones)
    S_NSCAL = 20
};
enum {
    F_DONE = 0,  // inner solve finished (kernels of the pass return at once)
    F_ITER,      // inner iterations of the current pass
    F_CONV,      // float64 residual below rtol
    F_SKIP,      // the current pass was skipped (already converged)
    F_ITER_TOT,  // inner iterations since the start of the solve
    F_PASSES,    // refinement passes since the start of the solve
    F_ITER1,     // inner iterations of the solve's first pass
    F_ERR,       // sticky device error bits (kErrVWindow)
    F_UNCONV,    // sticky count of pushes whose potential had not met rtol
    F_NFLAG = 12
};

// Device error bits (F_ERR): the assembly found the device step counter
// outside the window of conductor potentials (it then reads row 0).
constexpr int kErrVWindow = 1;

struct LevelDev {
    int NX, NY;
    float *u;          // correction (level 0: z at the start of the V-cycle)
    float *uo;         // pre-smoothed level from the down half-cycle (fine levels; = u on LDS levels)
    float *g;          // right-hand side (level 0: r)
    const uint8_t *fix;
};

struct CoarseArgs {
    int nlev;                      // levels handled in LDS
    int NX[kMaxLev], NY[kMaxLev];
    int off_u[kMaxLev], off_g[kMaxLev], off_f[kMaxLev]; // LDS byte offsets
    int off_s;                     // LDS scratch: one float per node of the first LDS level
    const uint8_t *fix[kMaxLev];   // global masks of those levels
    float *u_top;                  // global u of the first LDS level (output)
    const float *g_top;            // global g of the first LDS level (input)
    int px, py;
    int sweeps;                    // red-black pairs on the coarsest level
    int lds_bytes;
    const float *ainv;             // inverse of the coarsest level's operator (packed lower triangle), or null
    int dense_n;                   // its node count n when the coarsest level is solved exactly, else 0
    int off_p;                     // LDS: kCoarseWaves x n column partial sums of the exact solve
};

constexpr int kCoarseWaves = 16;   // wavefronts of the coarse kernel's work-group (1024 threads)
constexpr int kDenseMaxNodes = 768; // largest coarsest level given an explicit inverse (3 x 64 lanes x 4 floats)

// Packed lower triangle of a symmetric n x n matrix: row r holds columns
// 0 .. r padded with zeros to a multiple of 4 floats; its first float sits
// at tri_off(r) = sum over q < r of 4 (floor(q / 4) + 1).
__host__ __device__ inline long long tri_off(int r)
{
    const long long M = r >> 2, T = r & 3;
    return 4 * (M + 1) * (2 * M + T);
}

// Device descriptor of one instance.
struct Inst {
    Geom g;
    int nlev, lg, mg;
    LevelDev lev[kMaxLev];
    const uint8_t *node_cond, *cell_cond;
    double *phi, *b, *phi_prev;
    double *phi2;                  // second potential buffer of the Jacobi sweeps (solver 2)
    unsigned long long *rho[2];
    float *e, *p[2], *q;
    float *z;                      // preconditioned residual of the CG (level-0 u)
    // multigrid-preconditioned CG in the Chronopoulos-Gear form: residual
    // pair (lev[0].g, cg_r1), s = A p pair, w = A z
    float *cg_r1, *cg_s[2], *cg_w;
    float4 *E4;
    double *S;
    int *F;
    unsigned long long *surf;
    double qcharge;                // weight * 2^-32
    int charge_mode, charge_row, sjl, sjh;
    double sden;
    double rtol, eta_min;
    CoarseArgs coarse;
};

// Units of one launch: blocks boff[k] .. boff[k+1]-1 belong to unit id[k];
// grid kernels split a unit's blocks as bx[k] blocks across y.
struct Tab {
    int n;
    int id[kMaxUnits];
    int boff[kMaxUnits + 1];
    int bx[kMaxUnits];
};

struct HitLog {
    int32_t *rec;                  // capacity x 6 int32 (pic_hit layout)
    unsigned long long *count;
    long long capacity;
    int species_mask;
};

struct PushArgs {
    Geom g;
    int TX, TY, lx, ly, tiles_y, H, WX, WY;
    const uint8_t *cell_cond;
    const float4 *E4;              // per cell: (Ex,Ey) at corners 00,10 then 01,11
    int32_t *cell[2];              // both storage sets; info[7] selects the one in use
    float *ox[2], *oy[2], *vx[2], *vy[2];
    const int4 *table;             // (tile, start, end, 0) per block
    const long long *info;         // [1] table entries, [2 + set] slots, [7] set in use
    unsigned long long *rho;
    float qdt, dtf, hq;            // alpha dt, dt, alpha dt / 2 (float32)
    int box_i_top, box_j_lo, box_j_hi;
    int species, inst;
    unsigned long long *tally;     // 9 counters of this species
    unsigned long long *surf;      // trench-bottom hits per column, or null
    unsigned long long *iad;       // bottom-impact angle histogram (ions), or null
    HitLog log;
    const long long *step;         // device step counter (hit records)
    unsigned long long *fallbacks;
    int recycle_rows;              // > 0: lost ions of this species are recycled into rows 0 .. recycle_rows-1
                                   // (by k_recycle, after the push)
    unsigned recycle_key[2];
    double recycle_vth;
};

// Secondary electron emission of one instance (k_emit, k_emit_finish):
// the removals logged in the hit ring since the last call free electrons
// that are appended to species 0 (the set in use), after its binned slots.
struct SeeArgs {
    Geom g;
    const int32_t *rec;                 // hit ring, capacity x 6 int32 (pic_hit layout)
    const unsigned long long *log_count;// records written so far
    long long log_capacity;
    unsigned long long *misc;           // [0] records consumed, [1] slots asked this step,
                                        // [2] electrons appended, [3] dropped
    unsigned thresh[2];                 // floor(yield_s 2^24)
    double vth;
    unsigned key[2];
    int32_t *cell[2];                   // species 0, both storage sets; info[7] selects
    float *ox[2], *oy[2], *vx[2], *vy[2];
    long long *info;                    // species 0: [1] push blocks, [2 + set] slots,
                                        // [4] slots binned, [5] blocks of the binned slots, [7] set
    int4 *table;                        // species 0 push table
    long long capacity;
    int chunk;
    unsigned long long *rho;            // charge of species 0
};

struct BinArgs {
    int nx, ny;
    int lx, ly, tiles_y, ntiles, chunk;
    unsigned long long *bad;       // count of slots with a code outside the grid
    int32_t *cell[2];              // both storage sets: source info[7], destination the other
    float *ox[2], *oy[2], *vx[2], *vy[2];
    unsigned *counts, *offsets, *cursor, *boff;
    int4 *table;
    long long *info;               // [0] alive, [1] table entries, [2 + set] slots, [7] set in use
};

// Reduction partials: one float64 per block and quantity.
struct Part {
    double *p;
    int stride;
};

enum {
    OP_ASM = 0,      // after assembly: S_BB (or the source sum on fully periodic grids)
    OP_BB_PER,       // after the mean projection (fully periodic only): S_BB
    OP_SUM,          // S_SUM = t0
    OP_RR64_START,   // start residual: S_RR64, relres0, F_CONV, counters reset
    OP_RR64_PASS,    // residual after a pass (skipped passes keep their state)
    OP_INIT,         // inner start (inner stop ratio from the current residual)
    OP_PQ,           // S_PQ
    OP_UPDATE,       // S_RR, iteration count, inner stop test
    OP_RZ,           // rz rotation
    OP_UNUSED        // (the multigrid form's alpha and beta come from the level-0 down kernel)
};

// ---- launchers (pic_kernels.hip) --------------------------------------
// All launchers take the device Inst array and a Tab describing the units.
void launch_zero_u64(unsigned long long *p, long long n, hipStream_t s);
void launch_field(const Inst *I, const Tab &t, int zero_rho, hipStream_t s);
void launch_assemble(const Inst *I, const Tab &t, const double *Vtab, const long long *ctl,
                     int ninst, int vwin, Part pt, hipStream_t s);
void launch_project_mean(const Inst *I, const Tab &t, Part pt, hipStream_t s);
void launch_shift_mean(const Inst *I, const Tab &t, Part pt, hipStream_t s);
void launch_pin_shift(const Inst *I, const Tab &t, hipStream_t s);
void launch_set_guess(const Inst *I, const Tab &t, int kind, const double *guess, hipStream_t s);
void launch_extrapolate(const Inst *I, const Tab &t, int have_prev, hipStream_t s);
void launch_resid64(const Inst *I, const Tab &t, int after_pass, Part pt, hipStream_t s);
void launch_phi_update(const Inst *I, const Tab &t, hipStream_t s);
// `sweeps` Jacobi (an even count: the result lands in phi) or red-black
// Gauss-Seidel sweeps of the float64 system
void launch_sweeps(const Inst *I, const Tab &t, int jacobi, int sweeps, hipStream_t s);
void launch_init_red0(const Inst *I, const Tab &t, Part pt, hipStream_t s);
void launch_pupdate_Ap(const Inst *I, const Tab &t, int kold, int first, Part pt, hipStream_t s);
void launch_update_red0(const Inst *I, const Tab &t, int knew, Part pt, hipStream_t s);
void launch_coarse(const Inst *I, const Tab &t, int lds_bytes, const Tab &t0, Part pt, bool fuse, hipStream_t s);
// fused fine-level V-cycle halves (tables of 32 x 32 tiles of level l)
constexpr int kMgTileHost = 32;
// down: mode 0 level >= 1, mode 1 level 0 at the start of an inner pass,
// mode 2 level 0 after a CG step; par = buffer of the r / s pairs read
void launch_mg_down(const Inst *I, const Tab &t, int level, int mode, int par, Part pt, hipStream_t s);
void launch_mg_up(const Inst *I, const Tab &t, int level, int par, Part pt, hipStream_t s);
// levels l and l + 1 in one launch (table of level-(l+1) tiles); down or up
void launch_mg_pair(const Inst *I, const Tab &t, int level, bool down, hipStream_t s);
void launch_push(const PushArgs *A, const Tab &t, bool push, int unroll, int merge, size_t lds,
                 hipStream_t s);
void launch_rewind(const PushArgs *A, const Tab &t, hipStream_t s);
void launch_bin(const BinArgs *B, const Tab &tcount, const Tab &tscan, const Tab &ttable,
                hipStream_t s);
void launch_rho_sum(const unsigned long long *rho, long long n, unsigned long long *out,
                    hipStream_t s);
void launch_tick(long long *step, hipStream_t s);
// diagnostics: kinetic sums of one species' live particles (set in use) and
// the node-field energy of an instance, as kDiagBlocks partials each, then
// summed in block order into out[0] (kinetic) / out[0] (field)
void launch_kinetic(const PushArgs *A, int unit, double *part, double *out, hipStream_t s);
void launch_recycle(const PushArgs *A, const Tab &t, hipStream_t s);
// secondary electron emission: t has kEmitBlocks blocks per unit, t1 one
constexpr int kEmitBlocks = 32;
void launch_emit(const SeeArgs *A, const Tab &t, const Tab &t1, hipStream_t s);
void launch_field_energy(const Inst *I, int inst, double *part, double *out, hipStream_t s);
int bin_per_block();

// Dynamic LDS of the particle kernels: the tile + halo window of cell
// moments (16 B per cell), the class counters, and the corner fields of the
// tile + 1-cell frame (32 B per cell).
inline size_t push_lds_bytes(int TX, int TY, int H)
{
    const size_t mom = (size_t)(TX + 2 * H) * (TY + 2 * H) * 16 + kNClass * 4;
    // cell moments of the window, the corner fields of the tile + 1-cell frame,
    // the conductor map of the window + 1-cell frame
    return ((mom + 15) & ~(size_t)15) + (size_t)(TX + 2 * kFieldFrame) * (TY + 2 * kFieldFrame) * 32 +
           (size_t)(TX + 2 * H + 2) * (TY + 2 * H + 2);
}

} // namespace pic
