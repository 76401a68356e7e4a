/*
 * CPU oracle for the 2D electrostatic PIC cycle of Lin & Nishimura,
 * "Development of Particle-in-Cell Simulation in a Two Dimensional Trench
 * Geometry" (arXiv:1610.03918).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct reference code.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header or table with the HIP
 * library; both are written from the paper's equations independently.
 *
 * Units (Sec. II): lengths in Debye lengths, mesh spacing 1, time in
 * 1/omega_e, potential in T_e/e, density in n_0.
 *
 * Grid: nx x ny cells; x is the plate-normal axis (row index i), y the
 * plate-parallel axis (column j).  Nodes: NX = nx (periodic x) or nx+1,
 * NY = ny (periodic y) or ny+1.  Node (i,j) is stored at i*NY + j.  Cell
 * (i,j) spans nodes (i..i+1, j..j+1).  Particle cell codes are (i<<16)|j;
 * a negative code marks a removed particle.
 *
 * Floating point: built with -ffp-contract=off.  The "_f32" push rounds every
 * operation to float32 in the order written (for decisions that must match a
 * float32 device push bit for bit); the "_f64" push is the double-precision
 * reference of eqs. (1)-(4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXC 8
#define CI(c) ((int)(((uint32_t)(c)) >> 16))
#define CJ(c) ((int)(((uint32_t)(c)) & 0xFFFFu))

static int wrap(int a, int n) { a %= n; return a < 0 ? a + n : a; }

/* ------------------------------------------------------------------------
 * Geometry: which nodes carry a Dirichlet potential.
 * Sec. II: homogeneous Dirichlet at one electrode, RF Dirichlet at the other;
 * Sec. III.A: grounded walls; Sec. III.C: the trench is cut into the
 * electrode.  A node is Dirichlet when it lies on a bounded domain edge or
 * touches a solid (conductor) cell; it then takes that conductor's id.
 * Returns 0, or -1 when two different conductors meet at one node.
 * ---------------------------------------------------------------------- */
int or_node_cond(int nx, int ny, int px, int py, const uint8_t *cell_cond,
                 const int32_t *edge_cond, uint8_t *node_cond)
{
    int NX = px ? nx : nx + 1, NY = py ? ny : ny + 1;
    int bad = 0;
    for (int i = 0; i < NX; i++) {
        for (int j = 0; j < NY; j++) {
            int ids[6], k = 0;
            if (!px && i == 0) ids[k++] = edge_cond[0];
            if (!px && i == nx) ids[k++] = edge_cond[1];
            if (!py && j == 0) ids[k++] = edge_cond[2];
            if (!py && j == ny) ids[k++] = edge_cond[3];
            for (int di = -1; di <= 0; di++) {
                for (int dj = -1; dj <= 0; dj++) {
                    int ci = i + di, cj = j + dj;
                    if (px) ci = wrap(ci, nx); else if (ci < 0 || ci >= nx) continue;
                    if (py) cj = wrap(cj, ny); else if (cj < 0 || cj >= ny) continue;
                    int c = cell_cond[(size_t)ci * ny + cj];
                    if (c) {
                        int seen = 0;
                        for (int q = 0; q < k; q++) if (ids[q] == c) seen = 1;
                        if (!seen && k < 6) ids[k++] = c;
                    }
                }
            }
            int id = 0;
            for (int q = 0; q < k; q++) {
                if (ids[q] <= 0) continue;
                if (id && ids[q] != id) bad = 1;
                if (!id) id = ids[q];
            }
            node_cond[(size_t)i * NY + j] = (uint8_t)id;
        }
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------
 * Area (cloud-in-cell) weighting, integer form.  The paper does not state
 * its weighting; its PIC references use area weighting.  Offsets are
 * quantised to 16 bits per axis, u = floor(o * 2^16), and the four corner
 * weights (2^16-ux)(2^16-uy), ux(2^16-uy), (2^16-ux)uy, ux*uy sum to 2^32
 * exactly, so the node sums are exact integers, independent of order.
 * rho is accumulated (the caller clears it).
 * ---------------------------------------------------------------------- */
void or_deposit(int nx, int ny, int px, int py, int64_t n, const int32_t *cell,
                const float *ox, const float *oy, int64_t *rho)
{
    int NX = px ? nx : nx + 1, NY = py ? ny : ny + 1;
    (void)NX;
    const int64_t S = 65536;
    for (int64_t p = 0; p < n; p++) {
        int32_t c = cell[p];
        if (c < 0) continue;
        int i = CI(c), j = CJ(c);
        int64_t ux = (int64_t)floorf(ox[p] * 65536.0f);
        int64_t uy = (int64_t)floorf(oy[p] * 65536.0f);
        int i1 = px ? wrap(i + 1, nx) : i + 1;
        int j1 = py ? wrap(j + 1, ny) : j + 1;
        rho[(size_t)i * NY + j] += (S - ux) * (S - uy);
        rho[(size_t)i1 * NY + j] += ux * (S - uy);
        rho[(size_t)i * NY + j1] += (S - ux) * uy;
        rho[(size_t)i1 * NY + j1] += ux * uy;
    }
}

/* ------------------------------------------------------------------------
 * Right-hand side of eq. (5) written as -lap(phi) = n_i - n_e (q_i = e).
 * Free node: b = (N_i - N_e) * w * 2^-32 (+ static extra ion density), then
 * the Dirichlet neighbours' potentials are added in the order x-1, x+1,
 * y-1, y+1 (5-point stencil with unit spacing).  Dirichlet node: b = V.
 * Charge build-up (Sec. III.D): mode 1 adds a fixed density on one node row
 * over a y range; mode 2 adds half a particle (2^31 units) to each of the two
 * nodes of every trench-bottom face an ion has hit, on row charge_row.
 * ---------------------------------------------------------------------- */
void or_assemble(int nx, int ny, int px, int py, const uint8_t *node_cond,
                 const int64_t *rho_e, const int64_t *rho_i, double weight,
                 const double *V, int charge_mode, int charge_row,
                 const int64_t *surf, double static_density, int static_j_lo,
                 int static_j_hi, double *b)
{
    int NX = px ? nx : nx + 1, NY = py ? ny : ny + 1;
    double q = weight * ldexp(1.0, -32);
    for (int i = 0; i < NX; i++) {
        for (int j = 0; j < NY; j++) {
            size_t n = (size_t)i * NY + j;
            int c = node_cond[n];
            if (c) { b[n] = V[c]; continue; }
            int64_t Ni = rho_i[n];
            if (charge_mode == 2 && i == charge_row && surf) {
                int jl = py ? wrap(j - 1, ny) : j - 1;
                if (j < ny) Ni += surf[j] * ((int64_t)1 << 31);
                if (jl >= 0) Ni += surf[jl] * ((int64_t)1 << 31);
            }
            double r = (double)(Ni - rho_e[n]) * q;
            if (charge_mode == 1 && i == charge_row && j >= static_j_lo && j <= static_j_hi)
                r += static_density;
            int im = px ? wrap(i - 1, NX) : i - 1, ip = px ? wrap(i + 1, NX) : i + 1;
            int jm = py ? wrap(j - 1, NY) : j - 1, jp = py ? wrap(j + 1, NY) : j + 1;
            int cn;
            if ((cn = node_cond[(size_t)im * NY + j])) r += V[cn];
            if ((cn = node_cond[(size_t)ip * NY + j])) r += V[cn];
            if ((cn = node_cond[(size_t)i * NY + jm])) r += V[cn];
            if ((cn = node_cond[(size_t)i * NY + jp])) r += V[cn];
            b[n] = r;
        }
    }
}

/* y-neighbour / x-neighbour index helpers for the free-node operator */
static void nbrs(int i, int j, int NX, int NY, int px, int py, size_t out[4])
{
    int im = px ? wrap(i - 1, NX) : i - 1, ip = px ? wrap(i + 1, NX) : i + 1;
    int jm = py ? wrap(j - 1, NY) : j - 1, jp = py ? wrap(j + 1, NY) : j + 1;
    out[0] = (size_t)im * NY + j; out[1] = (size_t)ip * NY + j;
    out[2] = (size_t)i * NY + jm; out[3] = (size_t)i * NY + jp;
}

/* y = A x on free nodes, A = 4 - (sum of free neighbours); Dirichlet rows 0.
 * (The Dirichlet neighbours' values already sit in b.) */
static void apply_A(int NX, int NY, int px, int py, const uint8_t *fix,
                    const double *x, double *y)
{
    for (int i = 0; i < NX; i++)
        for (int j = 0; j < NY; j++) {
            size_t n = (size_t)i * NY + j;
            if (fix[n]) { y[n] = 0.0; continue; }
            size_t nb[4];
            nbrs(i, j, NX, NY, px, py, nb);
            double s = 4.0 * x[n];
            for (int k = 0; k < 4; k++) if (!fix[nb[k]]) s -= x[nb[k]];
            y[n] = s;
        }
}

/* ------------------------------------------------------------------------
 * Plain conjugate gradients in double precision on the free nodes (an
 * independent check of the direct solve; the paper itself iterates with
 * Gauss-Seidel / Jacobi, Sec. II).  phi holds the start on free nodes and
 * receives the Dirichlet values b on fixed nodes.  For a fully periodic grid
 * b must have zero mean; the result is shifted to zero mean.
 * Returns iterations, or -1 if not converged.
 * ---------------------------------------------------------------------- */
int or_cg(int NX, int NY, int px, int py, const uint8_t *node_cond,
          const double *b, double *phi, double rtol, int maxit, double *relres)
{
    size_t N = (size_t)NX * NY;
    double *r = calloc(N, sizeof(double)), *p = calloc(N, sizeof(double));
    double *q = calloc(N, sizeof(double));
    for (size_t n = 0; n < N; n++) if (node_cond[n]) phi[n] = b[n];
    apply_A(NX, NY, px, py, node_cond, phi, q);
    double bb = 0, rr = 0;
    for (size_t n = 0; n < N; n++) {
        if (node_cond[n]) continue;
        r[n] = b[n] - q[n];
        p[n] = r[n];
        bb += b[n] * b[n];
        rr += r[n] * r[n];
    }
    if (bb == 0) bb = 1;
    int it = 0, ok = 0;
    for (; it < maxit; it++) {
        if (sqrt(rr / bb) <= rtol) { ok = 1; break; }
        apply_A(NX, NY, px, py, node_cond, p, q);
        double pq = 0;
        for (size_t n = 0; n < N; n++) if (!node_cond[n]) pq += p[n] * q[n];
        double a = rr / pq, rr2 = 0;
        for (size_t n = 0; n < N; n++) {
            if (node_cond[n]) continue;
            phi[n] += a * p[n];
            r[n] -= a * q[n];
            rr2 += r[n] * r[n];
        }
        double be = rr2 / rr;
        rr = rr2;
        for (size_t n = 0; n < N; n++) if (!node_cond[n]) p[n] = r[n] + be * p[n];
    }
    if (!ok && sqrt(rr / bb) <= rtol) ok = 1;
    if (px && py) {
        double m = 0;
        for (size_t n = 0; n < N; n++) m += phi[n];
        m /= (double)N;
        for (size_t n = 0; n < N; n++) phi[n] -= m;
    }
    if (relres) *relres = sqrt(rr / bb);
    free(r); free(p); free(q);
    return ok ? it : -1;
}

/* ------------------------------------------------------------------------
 * E = -grad(phi) at the nodes (Sec. II).  Central differences inside.  At a
 * Dirichlet node, along each axis: if exactly one neighbour exists and is a
 * free node, the two-point one-sided difference toward it; otherwise, if both
 * neighbours exist, the central difference (zero along an equipotential
 * conductor: tangential E vanishes at a conducting wall, Sec. III.A); at a
 * domain edge the two-point difference with the one existing neighbour.
 * ---------------------------------------------------------------------- */
static double axis_E(double phm, double ph0, double php, int has_m, int has_p,
                     int free_m, int free_p, int fixed_here)
{
    if (!fixed_here) return -(php - phm) * 0.5;
    if (has_m && has_p) {
        if (free_p && !free_m) return -(php - ph0);
        if (free_m && !free_p) return -(ph0 - phm);
        return -(php - phm) * 0.5;
    }
    if (has_p) return -(php - ph0);
    if (has_m) return -(ph0 - phm);
    return 0.0;
}

void or_field(int NX, int NY, int px, int py, const uint8_t *node_cond,
              const double *phi, double *Ex, double *Ey)
{
    for (int i = 0; i < NX; i++)
        for (int j = 0; j < NY; j++) {
            size_t n = (size_t)i * NY + j;
            int fixed = node_cond[n] != 0;
            int hm = px || i > 0, hp = px || i < NX - 1;
            int im = px ? wrap(i - 1, NX) : i - 1, ip = px ? wrap(i + 1, NX) : i + 1;
            double a = hm ? phi[(size_t)im * NY + j] : 0.0;
            double c = hp ? phi[(size_t)ip * NY + j] : 0.0;
            int fm = hm && !node_cond[(size_t)im * NY + j];
            int fp = hp && !node_cond[(size_t)ip * NY + j];
            Ex[n] = axis_E(a, phi[n], c, hm, hp, fm, fp, fixed);
            int gm = py || j > 0, gp = py || j < NY - 1;
            int jm = py ? wrap(j - 1, NY) : j - 1, jp = py ? wrap(j + 1, NY) : j + 1;
            double d = gm ? phi[(size_t)i * NY + jm] : 0.0;
            double e = gp ? phi[(size_t)i * NY + jp] : 0.0;
            int hm2 = gm && !node_cond[(size_t)i * NY + jm];
            int hp2 = gp && !node_cond[(size_t)i * NY + jp];
            Ey[n] = axis_E(d, phi[n], e, gm, gp, hm2, hp2, fixed);
        }
}

/* ------------------------------------------------------------------------
 * Gather + leapfrog push + wall/conductor test, eqs. (1)-(4).
 *   E_p   = bilinear interpolation of the corner fields, weights
 *           (1-ox)(1-oy), ox(1-oy), (1-ox)oy, ox*oy, summed in that order
 *   v    += (alpha dt) E_p          (v^{n+1/2} = v^{n-1/2} + alpha E^n dt)
 *   D     = v dt,  o' = o + D       (x^{n+1} = x^n + v^{n+1/2} dt)
 * The straight segment o -> o' is walked cell by cell: at each step the
 * earlier of the next x face and the next y face is crossed, compared as
 * (fx + kx)|Dy| <= (fy + ky)|Dx| (ties cross x first).  Periodic axes wrap.
 * Entering a solid cell or leaving a bounded axis removes the particle; the
 * hit is classified by the crossing direction (0 +x, 1 -x, 2 +y, 3 -y) plus 4
 * when the last cell occupied lies in the trench box.  Class 8 marks a
 * non-finite or runaway (>= 1e6 cells) displacement.  The removed particle's
 * code becomes -1 - class.  An ion leaving through +x inside the box hits the
 * trench bottom and, if surf is given, bumps surf[j] of that cell.
 * tally has 9 entries.  T is float (every operation rounded to float32) or
 * double; the state arrays have the same type.
 * ---------------------------------------------------------------------- */
/* ------------------------------------------------------------------------
 * Ion recycling (Sec. III.A, III.C): an ion lost at a wall is replaced by a
 * thermal ion in the bulk plasma, the ionisation of the ambient gas, only in
 * the bulk rows 0 .. rows-1.  The new ion's cell, offsets and velocity come
 * from a counter-based generator, Philox4x32-10 (Salmon, Moraes, Dror and
 * Shaw, SC 2011), keyed by the run's seed and counting on (step, bits of the
 * lost ion's v_x after the kick, bits of its offsets before the move), so
 * they do not depend on the order in which particles are stored:
 *   r  = Philox(ctr, key), r' = Philox(ctr, key + (0, 1))
 *   i  = (r0 >> 8) * rows >> 24,  j = (r1 >> 8) * ny >> 24   (exact integers)
 *   ox = (r2 >> 8) 2^-24,  oy = (r3 >> 8) 2^-24              (exact floats)
 *   (vx, vy) = vth sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v) in double,
 *   u = ((r'0 >> 8) + 1) 2^-24, v = (r'1 >> 8) 2^-24        (Box-Muller)
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t rows;                 /* 0: no recycling */
    uint32_t k0, k1;
    double vth;                   /* ion thermal speed per component */
    int64_t step;                 /* step being pushed */
} or_recycle;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t f32_bits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

void or_recycled_ion(const or_recycle *rc, float ux, float ox0, float oy0, int ny, int32_t *code,
                     float *ox, float *oy, double *vx, double *vy)
{
    uint32_t ctr[4] = {(uint32_t)rc->step, f32_bits(ux), f32_bits(ox0), f32_bits(oy0)};
    uint32_t key[2] = {rc->k0, rc->k1}, r[4], q[4];
    or_philox4x32_10(ctr, key, r);
    key[1] += 1u;
    or_philox4x32_10(ctr, key, q);
    uint32_t i = (uint32_t)(((uint64_t)(r[0] >> 8) * (uint32_t)rc->rows) >> 24);
    uint32_t j = (uint32_t)(((uint64_t)(r[1] >> 8) * (uint32_t)ny) >> 24);
    *code = (int32_t)((i << 16) | j);
    *ox = (float)(r[2] >> 8) * 0x1p-24f;
    *oy = (float)(r[3] >> 8) * 0x1p-24f;
    double u = (double)((q[0] >> 8) + 1u) * 0x1p-24, v = (double)(q[1] >> 8) * 0x1p-24;
    double rad = sqrt(-2.0 * log(u)), ang = 6.283185307179586 * v;
    *vx = rc->vth * rad * cos(ang);
    *vy = rc->vth * rad * sin(ang);
}

/* Optional record of every removal of the push: (class, last cell occupied
 * as a packed code, bits of the kicked float32 velocity), cap rows. */
typedef struct {
    int64_t cap, n;
    int32_t *rec;                 /* cap x 4 */
} or_hits;

static void hit_record(or_hits *h, int cls, int ci, int cj, float ux, float uy)
{
    if (!h) return;
    if (h->n < h->cap) {
        int32_t *r = h->rec + 4 * h->n;
        r[0] = cls;
        r[1] = (int32_t)(((uint32_t)ci << 16) | (uint32_t)cj);
        memcpy(&r[2], &ux, 4);
        memcpy(&r[3], &uy, 4);
    }
    h->n++;
}

#define PUSH_BODY(T, FLOOR)                                                          \
    int NY = py ? ny : ny + 1;                                                       \
    T qdt = (T)(alpha * dt), dtt = (T)dt;                                            \
    int64_t lost = 0;                                                                \
    for (int64_t p = 0; p < n; p++) {                                                \
        int32_t c = cell[p];                                                         \
        if (c < 0) continue;                                                         \
        int i = CI(c), j = CJ(c);                                                    \
        int i1 = px ? wrap(i + 1, nx) : i + 1;                                       \
        int j1 = py ? wrap(j + 1, ny) : j + 1;                                       \
        size_t n00 = (size_t)i * NY + j, n10 = (size_t)i1 * NY + j;                  \
        size_t n01 = (size_t)i * NY + j1, n11 = (size_t)i1 * NY + j1;                \
        T x0 = ox[p], y0 = oy[p];                                                    \
        T wx0 = (T)1 - x0, wy0 = (T)1 - y0;                                          \
        T w00 = wx0 * wy0, w10 = x0 * wy0, w01 = wx0 * y0, w11 = x0 * y0;            \
        T ex = w00 * (T)Ex[n00];                                                     \
        ex = ex + w10 * (T)Ex[n10];                                                  \
        ex = ex + w01 * (T)Ex[n01];                                                  \
        ex = ex + w11 * (T)Ex[n11];                                                  \
        T ey = w00 * (T)Ey[n00];                                                     \
        ey = ey + w10 * (T)Ey[n10];                                                  \
        ey = ey + w01 * (T)Ey[n01];                                                  \
        ey = ey + w11 * (T)Ey[n11];                                                  \
        T ux = vx[p] + qdt * ex;                                                     \
        T uy = vy[p] + qdt * ey;                                                     \
        T Dx = ux * dtt, Dy = uy * dtt;                                              \
        T x1 = x0 + Dx, y1 = y0 + Dy;                                                \
        T fsx = FLOOR(x1), fsy = FLOOR(y1);                                          \
        vx[p] = ux; vy[p] = uy;                                                      \
        if (!(fabs((double)fsx) < 1.0e6 && fabs((double)fsy) < 1.0e6)) {            \
            cell[p] = -1 - 8; lost++;                                                \
            if (tally) tally[8]++;                                                   \
            hit_record(hits, 8, i, j, (float)ux, (float)uy);                         \
            continue;                                                                \
        }                                                                            \
        int sx = (int)fsx, sy = (int)fsy;                                            \
        int ci = i, cj = j, dead = -1;                                               \
        if (sx != 0 || sy != 0) {                                                    \
            T ax = Dx < 0 ? -Dx : Dx, ay = Dy < 0 ? -Dy : Dy;                         \
            T fx = sx > 0 ? (T)1 - x0 : x0, fy = sy > 0 ? (T)1 - y0 : y0;            \
            int nxs = abs(sx), nys = abs(sy), kx = 0, ky = 0;                        \
            int di = sx > 0 ? 1 : -1, dj = sy > 0 ? 1 : -1;                          \
            while (kx < nxs || ky < nys) {                                           \
                int gox;                                                             \
                if (ky >= nys) gox = 1;                                              \
                else if (kx >= nxs) gox = 0;                                         \
                else gox = ((fx + (T)kx) * ay <= (fy + (T)ky) * ax);                 \
                int ni = ci, nj = cj, dir;                                           \
                if (gox) { ni = ci + di; kx++; dir = di > 0 ? 0 : 1; }               \
                else { nj = cj + dj; ky++; dir = dj > 0 ? 2 : 3; }                   \
                int out = 0;                                                         \
                if (px) ni = wrap(ni, nx); else if (ni < 0 || ni >= nx) out = 1;     \
                if (py) nj = wrap(nj, ny); else if (nj < 0 || nj >= ny) out = 1;     \
                if (!out && cell_cond[(size_t)ni * ny + nj]) out = 1;                \
                if (out) {                                                           \
                    int inbox = ci >= box_i_top && cj >= box_j_lo && cj < box_j_hi;  \
                    dead = dir + 4 * inbox;                                          \
                    break;                                                           \
                }                                                                    \
                ci = ni; cj = nj;                                                    \
            }                                                                        \
        }                                                                            \
        if (dead >= 0) {                                                             \
            cell[p] = -1 - dead;                                                     \
            lost++;                                                                  \
            if (tally) tally[dead]++;                                                \
            if (surf && dead == 4) surf[cj]++;                                       \
            hit_record(hits, dead, ci, cj, (float)ux, (float)uy);                    \
            if (rc && rc->rows > 0) {                                                \
                int32_t code; float nox, noy; double nvx, nvy;                       \
                or_recycled_ion(rc, (float)ux, (float)x0, (float)y0, ny, &code,      \
                             &nox, &noy, &nvx, &nvy);                                \
                cell[p] = code; ox[p] = (T)nox; oy[p] = (T)noy;                      \
                vx[p] = (T)nvx; vy[p] = (T)nvy;                                      \
            }                                                                        \
            continue;                                                                \
        }                                                                            \
        T nxo = x1 - (T)sx, nyo = y1 - (T)sy;                                        \
        ox[p] = below_one_##T(nxo);                                                  \
        oy[p] = below_one_##T(nyo);                                                  \
        cell[p] = (int32_t)(((uint32_t)ci << 16) | (uint32_t)cj);                    \
    }                                                                                \
    return lost;

/* the in-cell offset is kept in [0, 1): a value that rounds up to 1 (from a
 * tiny negative o' - floor(o')) becomes the largest float below 1 */
static float below_one_float(float o) { return o >= 1.0f ? nextafterf(1.0f, 0.0f) : o; }
static double below_one_double(double o) { return o >= 1.0 ? nextafter(1.0, 0.0) : o; }

int64_t or_push_f32(int nx, int ny, int px, int py, const uint8_t *cell_cond,
                    int box_i_top, int box_j_lo, int box_j_hi, double dt, double alpha,
                    const double *Ex, const double *Ey, int64_t n, int32_t *cell,
                    float *ox, float *oy, float *vx, float *vy, int64_t *tally,
                    int64_t *surf, const or_recycle *rc, or_hits *hits)
{
    PUSH_BODY(float, floorf)
}

int64_t or_push_f64(int nx, int ny, int px, int py, const uint8_t *cell_cond,
                    int box_i_top, int box_j_lo, int box_j_hi, double dt, double alpha,
                    const double *Ex, const double *Ey, int64_t n, int32_t *cell,
                    double *ox, double *oy, double *vx, double *vy, int64_t *tally,
                    int64_t *surf, const or_recycle *rc, or_hits *hits)
{
    PUSH_BODY(double, floor)
}

/* ------------------------------------------------------------------------
 * Start of the leapfrog (the paper does not state it): velocities are moved
 * back half a step, v^{-1/2} = v^0 - (alpha dt / 2) E^0(x^0).
 * ---------------------------------------------------------------------- */
#define REWIND_BODY(T)                                                               \
    int NY = py ? ny : ny + 1;                                                       \
    T h = (T)(0.5 * alpha * dt);                                                     \
    for (int64_t p = 0; p < n; p++) {                                                \
        int32_t c = cell[p];                                                         \
        if (c < 0) continue;                                                         \
        int i = CI(c), j = CJ(c);                                                    \
        int i1 = px ? wrap(i + 1, nx) : i + 1;                                       \
        int j1 = py ? wrap(j + 1, ny) : j + 1;                                       \
        size_t n00 = (size_t)i * NY + j, n10 = (size_t)i1 * NY + j;                  \
        size_t n01 = (size_t)i * NY + j1, n11 = (size_t)i1 * NY + j1;                \
        T x0 = ox[p], y0 = oy[p];                                                    \
        T wx0 = (T)1 - x0, wy0 = (T)1 - y0;                                          \
        T w00 = wx0 * wy0, w10 = x0 * wy0, w01 = wx0 * y0, w11 = x0 * y0;            \
        T ex = w00 * (T)Ex[n00];                                                     \
        ex = ex + w10 * (T)Ex[n10];                                                  \
        ex = ex + w01 * (T)Ex[n01];                                                  \
        ex = ex + w11 * (T)Ex[n11];                                                  \
        T ey = w00 * (T)Ey[n00];                                                     \
        ey = ey + w10 * (T)Ey[n10];                                                  \
        ey = ey + w01 * (T)Ey[n01];                                                  \
        ey = ey + w11 * (T)Ey[n11];                                                  \
        vx[p] = vx[p] - h * ex;                                                      \
        vy[p] = vy[p] - h * ey;                                                      \
    }

void or_rewind_f32(int nx, int ny, int px, int py, double dt, double alpha,
                   const double *Ex, const double *Ey, int64_t n, const int32_t *cell,
                   const float *ox, const float *oy, float *vx, float *vy)
{
    REWIND_BODY(float)
}

void or_rewind_f64(int nx, int ny, int px, int py, double dt, double alpha,
                   const double *Ex, const double *Ey, int64_t n, const int32_t *cell,
                   const double *ox, const double *oy, double *vx, double *vy)
{
    REWIND_BODY(double)
}

/* ------------------------------------------------------------------------
 * Secondary electron emission at the trench surfaces.  The paper names it
 * as future work (Sec. IV: emission through ion and through electron
 * bombardment) and gives no yield model.  Reading taken: a particle of
 * species s removed at a trench surface (the bottom, class 4; the
 * sidewalls, classes 6 and 7) frees one electron with the constant
 * probability yield_s.  The electron starts in the cell the particle last
 * occupied, on the struck face (normal offset at the face: the largest float
 * below 1 on a cell's high side, 0 on its low side), uniformly along it, and
 * leaves the surface with a flux-weighted half-Maxwellian of thermal speed
 * vth: normal speed vth sqrt(-2 ln u) away from the wall, tangential
 * velocity vth sqrt(-2 ln u') cos(2 pi u'').  Its velocity is taken as the
 * half-step velocity of the step that created it (as for recycled ions).
 * Draws: Philox4x32-10 (Salmon et al., SC 2011) keyed by (k0, k1), counter
 * (step, packed cell, bits of the kicked float32 velocity (ux, uy)):
 *   r = Philox(ctr, (k0, k1)):     emitted iff (r0 >> 8) < thresh_s
 *                                  (thresh_s = floor(yield_s 2^24));
 *                                  along-face offset (r1 >> 8) 2^-24
 *   q = Philox(ctr, (k0, k1 + 1)): u = ((q0 >> 8) + 1) 2^-24,
 *                                  u' = ((q1 >> 8) + 1) 2^-24, u'' = (q2 >> 8) 2^-24
 * in double, the velocity rounded to float.  Input: nh removals (species
 * and a 4-word record each, as or_hits writes them); output: the emitted
 * electrons (at most nh).  Returns their number.
 * ---------------------------------------------------------------------- */
int64_t or_emit(int64_t nh, const int32_t *species, const int32_t *rec, int64_t step, uint32_t k0, uint32_t k1,
                const uint32_t *thresh, double vth, int32_t *cell, float *ox, float *oy, float *vx, float *vy)
{
    int64_t m = 0;
    const float below1 = nextafterf(1.0f, 0.0f);
    for (int64_t h = 0; h < nh; h++) {
        const int32_t *r4 = rec + 4 * h;
        const int cls = r4[0];
        if (cls != 4 && cls != 6 && cls != 7) continue;
        const int s = species[h];
        if (s < 0 || s > 1 || thresh[s] == 0) continue;
        uint32_t ctr[4] = {(uint32_t)step, (uint32_t)r4[1], (uint32_t)r4[2], (uint32_t)r4[3]};
        uint32_t key[2] = {k0, k1}, r[4], q[4];
        or_philox4x32_10(ctr, key, r);
        if ((r[0] >> 8) >= thresh[s]) continue;
        key[1] += 1u;
        or_philox4x32_10(ctr, key, q);
        const float a = (float)(r[1] >> 8) * 0x1p-24f;
        const double u1 = (double)((q[0] >> 8) + 1u) * 0x1p-24, u2 = (double)((q[1] >> 8) + 1u) * 0x1p-24;
        const double u3 = (double)(q[2] >> 8) * 0x1p-24;
        const double vn = vth * sqrt(-2.0 * log(u1));
        const double vt = vth * sqrt(-2.0 * log(u2)) * cos(6.283185307179586 * u3);
        cell[m] = r4[1];
        if (cls == 4) {                 /* +x face (the bottom): back along -x */
            ox[m] = below1; oy[m] = a; vx[m] = (float)(-vn); vy[m] = (float)vt;
        } else if (cls == 6) {          /* +y face: back along -y */
            ox[m] = a; oy[m] = below1; vx[m] = (float)vt; vy[m] = (float)(-vn);
        } else {                        /* -y face: back along +y */
            ox[m] = a; oy[m] = 0.0f; vx[m] = (float)vt; vy[m] = (float)vn;
        }
        m++;
    }
    return m;
}
