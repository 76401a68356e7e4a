// Internal interface between the gfx950 kernels (pic_kernels.hip) and the
// host runtime behind the C ABI (pic_runtime.cpp).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kMaxLev = 16;
constexpr int kNClass = 9;
constexpr int kGridBX = 64;      // grid kernels: 64 x 4 threads over (y, x) nodes
constexpr int kGridBY = 4;
constexpr int kPushThreads = 256;

struct Geom {
    int nx, ny;     // cells
    int NX, NY;     // nodes
    int px, py;     // periodic axes
};

// Slots of the float64 scalar block and the int flag block of the solver.
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
    S_NSCAL = 16
};
enum { F_DONE = 0, F_ITER, F_NFLAG = 8 };

// Reduction bookkeeping: one partial per block, one counter per reduction.
struct Red {
    double *part;      // partial sums, stride max_blocks per quantity
    int stride;
    unsigned *count;   // arrival counter (reset by the last block)
    double *S;         // float64 scalars
    int *F;            // int flags / counters
};

struct LevelDev {
    int NX, NY;
    float *u;          // correction (level 0: z)
    float *g;          // right-hand side (level 0: r)
    const uint8_t *fix;
};

struct CoarseArgs {
    int nlev;                      // levels handled in LDS
    int NX[kMaxLev], NY[kMaxLev];
    int off_u[kMaxLev], off_g[kMaxLev], off_f[kMaxLev]; // LDS byte offsets
    const uint8_t *fix[kMaxLev];   // global masks of those levels
    float *u_top;                  // global u of the first LDS level (output)
    const float *g_top;            // global g of the first LDS level (input)
    int px, py;
    int sweeps;                    // red-black pairs on the coarsest level
    int lds_bytes;
};

struct VTab {
    double v[8];                   // conductor potentials at the assembly time
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
    int32_t *cell;
    float *ox, *oy, *vx, *vy;
    const int4 *table;             // (tile, start, end, 0) per block
    const long long *info;         // [1] = number of table entries
    unsigned long long *rho;
    float qdt, dtf;
    int box_i_top, box_j_lo, box_j_hi;
    int species;
    unsigned long long *tally;     // 9 counters of this species
    unsigned long long *surf;      // trench-bottom hits per column, or null
    HitLog log;
    int step;
    unsigned long long *fallbacks;
};

struct BinArgs {
    int nx, ny;
    int lx, ly, tiles_y, ntiles, chunk;
    unsigned long long *bad;       // count of slots with a code outside the grid
    const int32_t *cell;
    const float *ox, *oy, *vx, *vy;
    int32_t *cell2;
    float *ox2, *oy2, *vx2, *vy2;
    const long long *slots;        // device slot count of the source set
    unsigned *counts, *offsets, *cursor, *boff;
    int4 *table;
    long long *info;               // [0] alive, [1] table entries, [2 + set] slots of each set
    int dst;                       // destination set
};

// ---- launchers (pic_kernels.hip) --------------------------------------
void launch_zero_u64(unsigned long long *p, long long n, hipStream_t s);
void launch_field(const Geom &g, const uint8_t *node_cond, const double *phi, float4 *E4,
                  unsigned long long *rho0, unsigned long long *rho1, hipStream_t s);
void launch_assemble(const Geom &g, const uint8_t *node_cond, const uint8_t *fix0,
                     const long long *rho_e, const long long *rho_i, double q,
                     const VTab &V, int charge_mode, int charge_row,
                     const unsigned long long *surf, double static_density, int sj_lo,
                     int sj_hi, double *b, double *phi, Red red, hipStream_t s);
void launch_project_mean(const Geom &g, const uint8_t *fix0, double *b, Red red, hipStream_t s);
void launch_shift_mean(const Geom &g, double *phi, Red red, hipStream_t s);
void launch_pin_shift(const Geom &g, double *phi, Red red, hipStream_t s);
void launch_extrapolate(const Geom &g, const uint8_t *fix0, double *phi, double *prev, int have_prev,
                        hipStream_t s);
void launch_set_guess(const Geom &g, const uint8_t *fix0, int kind, const double *guess,
                      double *phi, hipStream_t s);
void launch_resid64(const Geom &g, const uint8_t *fix0, const double *b, const double *phi,
                    float *r, Red red, hipStream_t s);
void launch_phi_update(const Geom &g, const uint8_t *fix0, const float *e, double *phi,
                       hipStream_t s);
void launch_init_red0(const Geom &g, const LevelDev &L0, float *e, double eta2, int mg,
                      Red red, hipStream_t s);
void launch_pupdate_Ap(const Geom &g, const LevelDev &L0, const float *p_old, float *p_new,
                       float *q, int first, Red red, hipStream_t s);
void launch_update_red0(const Geom &g, const LevelDev &L0, const float *p, const float *q,
                        float *e, int mg, Red red, hipStream_t s);
void launch_smooth(const Geom &g, const LevelDev &L, int color, int level0_rz, Red red,
                   hipStream_t s);
void launch_restrict(const Geom &g, const LevelDev &F, const LevelDev &Cc, const int *done,
                     hipStream_t s);
void launch_prolong_black(const Geom &g, const LevelDev &F, const LevelDev &Cc, const int *done,
                          hipStream_t s);
void launch_coarse(const CoarseArgs &a, const int *done, hipStream_t s);
void launch_push(const PushArgs &a, int max_blocks, bool push, int unroll, int merge,
                 hipStream_t s);
void launch_rewind(const Geom &g, const float4 *E4, const int32_t *cell, const float *ox,
                   const float *oy, float *vx, float *vy, long long n, const long long *slots,
                   float hq, hipStream_t s);
void launch_bin(const BinArgs &a, long long max_slots, hipStream_t s);
void launch_rho_sum(const unsigned long long *rho, long long n, unsigned long long *out,
                    hipStream_t s);

} // namespace pic
