/*
 * FP64 CPU oracle of one explicit time step of the Lagrangian-particle (LP)
 * method for granular flow with mu(I) rheology (Zepeda & Samulyak,
 * "Computational Model for Granular Flows based on the Lagrangian Particle
 * Method", arXiv:2206.14061).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the HIP
 * library is checked against.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the library never does.  It shares
 * no code, header, table or constant generator with the HIP sources.
 *
 * Everything is float64, built with -ffp-contract=off.  OpenMP (when
 * enabled) only distributes independent particles; results do not depend
 * on the thread count.
 *
 * What each part follows:
 *   mirrors ............ Sec. 3.1 step 9, solid-boundary (mirror) particles
 *   neighbours ......... Sec. 3.1 step 5 (all particles within radius R)
 *   stencil order ...... Sec. 3.1 step 6 (top entries cover all octants,
 *                        then ascending distance), truncated to m_max
 *   ghosts ............. Sec. 3.1 steps 5 and 9 (free-boundary ghosts)
 *   fit ................ Sec. 3.1 step 7 (2nd-order Taylor rows, least
 *                        squares by QR), extended to 3D with 9 unknowns
 *   closure ............ Sec. 2.2 (strain rate, shear rate, inertial
 *                        number, mu(I), alignment) and Sec. 2.2.1 (regime
 *                        transitions, eq. EOS2)
 *   RHS ................ Sec. 2.1 momentum and mass equations with
 *                        sigma = -P delta + eta gamma_dot ("Form E")
 *   Form M ............. Sec. 2.3 / Sec. 3.1 step 8 printed update with
 *                        M, N, S and a sign-corrected R (cross-check only)
 *   update ............. Sec. 3.1 step 8 (explicit Euler for V and u) and
 *                        step 10 (trapezoidal particle displacement)
 *
 * Parameter record (per system, 16 doubles):
 *   rho_s d mu_s mu_2 I0 phi_c phi_min phi_max alpha beta gx gy gz h R wall_z
 * Config record (6 doubles):
 *   m_max ghost_margin(*h) phi_ghost_frac fallback_tol weight(0 unit,1 gauss)
 *   wall_pressure(0 mirror P(phi_src), 1 plus the hydrostatic weight)
 *   fit_order(2 quadratic, 3 cubic)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { P_RHO, P_D, P_MUS, P_MU2, P_I0, P_PHIC, P_PHIMIN, P_PHIMAX, P_ALPHA,
       P_BETA, P_GX, P_GY, P_GZ, P_H, P_R, P_WALL, P_XLO, P_YLO, P_LX, P_LY,
       P_NPRM };
enum { C_MMAX, C_GMARGIN, C_PHIG, C_FTOL, C_WEIGHT, C_WALLP, C_ORDER, C_MINREAL, C_NCFG };

#define NC 9          /* unknowns of the 2nd-order 3D fit            */
#define NC3 19        /* unknowns of the 3rd-order (cubic) 3D fit    */
#define MAXROWS 256   /* rows the oracle can hold for one stencil    */

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of later parallel regions (timing runs at 1 thread and at all
 * cores); 0 or less restores the count the process started with. */
void orc_set_threads(int t)
{
#ifdef _OPENMP
    static int initial = 0;
    if (!initial) initial = omp_get_max_threads();
    omp_set_num_threads(t > 0 ? t : initial);
#else
    (void)t;
#endif
}

/* ------------------------------------------------------------------ */
/* Morton order of the particles of each system.                       */
/* ------------------------------------------------------------------ */

static uint64_t spread3(uint64_t v)
{
    /* bit k of v goes to bit 3k (plain loop, no magic constants) */
    uint64_t r = 0;
    for (int k = 0; k < 21; ++k)
        r |= ((v >> k) & 1ull) << (3 * k);
    return r;
}

/* Periodic axes (Sec. 3.1, boundary conditions): an axis with period
 * L > 0 over [lo, lo + L) identifies x with x + L.  wrap_coord maps a
 * coordinate within one period of the box into it (one correction);
 * image_coord gives the copy of x_j nearest to x_i (x_j - L when
 * x_j - x_i > L/2, x_j + L when below -L/2). */
static double wrap_coord(double x, double lo, double L)
{
    if (L > 0.0) {
        if (x >= lo + L) return x - L;
        if (x < lo) return x + L;
    }
    return x;
}

static double image_coord(double xj, double xi, double L)
{
    if (L > 0.0) {
        double d = xj - xi;
        if (d > 0.5 * L) return xj - L;
        if (d < -0.5 * L) return xj + L;
    }
    return xj;
}

/* cells along a periodic axis: floor(L / c) (at least 1) of edge L / n */
static int64_t periodic_cells(double L, double ic)
{
    int64_t nc = (int64_t)(L * ic);
    return nc < 1 ? 1 : nc;
}

typedef struct { uint64_t key; int64_t idx; } KeyIdx;

static int cmp_keyidx(const void* a, const void* b)
{
    const KeyIdx* p = (const KeyIdx*)a;
    const KeyIdx* q = (const KeyIdx*)b;
    if (p->key != q->key) return p->key < q->key ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

/* Cell edge c = R (1 + skin) (1 + 2^-20), origin (min x, min y,
 * min(min z, wall - R)) per system; cell coordinate floor((x - origin)/c)
 * computed as (x - origin) * (1/c); key = bit interleave (x -> 3k,
 * y -> 3k+1, z -> 3k+2).  A periodic axis starts at its box and has
 * n = floor(L/c) cells: coordinate (wrap(x) - lo) * (n / L), clamped to
 * [0, n - 1].  Particles are ordered by (key, old index) inside
 * each system.  perm[new] = old.  Returns -1 if a cell coordinate needs
 * more than 21 bits.  (The order only affects which particle gets which
 * id; skin is the neighbour-list margin of the GPU library, whose cells
 * have this edge.) */
int orc_sort(int64_t n, int32_t n_sys, const int64_t* off, const double* prm,
             double skin, const double* x, const double* y, const double* z,
             int32_t* perm, uint64_t* keys)
{
    KeyIdx* t = (KeyIdx*)malloc(sizeof(KeyIdx) * (size_t)(n > 0 ? n : 1));
    int bad = 0;
    for (int s = 0; s < n_sys; ++s) {
        const double* p = prm + (size_t)s * P_NPRM;
        int64_t a = off[s], b = off[s + 1];
        if (b <= a) continue;
        double x0 = x[a], y0 = y[a], z0 = z[a];
        for (int64_t i = a; i < b; ++i) {
            if (x[i] < x0) x0 = x[i];
            if (y[i] < y0) y0 = y[i];
            if (z[i] < z0) z0 = z[i];
        }
        double zl = p[P_WALL] - p[P_R];
        if (zl < z0) z0 = zl;
        double c = (p[P_R] * (1.0 + skin)) * (1.0 + 1.0 / 1048576.0);
        double ic = 1.0 / c;
        double Lx = p[P_LX], Ly = p[P_LY];
        double icx = ic, icy = ic;
        int64_t npx = 0, npy = 0;
        if (Lx > 0.0) { x0 = p[P_XLO]; npx = periodic_cells(Lx, ic); icx = (double)npx / Lx; }
        if (Ly > 0.0) { y0 = p[P_YLO]; npy = periodic_cells(Ly, ic); icy = (double)npy / Ly; }
        for (int64_t i = a; i < b; ++i) {
            double xw = wrap_coord(x[i], p[P_XLO], Lx);
            double yw = wrap_coord(y[i], p[P_YLO], Ly);
            double fx = (xw - x0) * icx, fy = (yw - y0) * icy,
                   fz = (z[i] - z0) * ic;
            uint64_t cx, cy, cz = (uint64_t)fz;
            if (Lx > 0.0) {
                int64_t t = (int64_t)fx;
                cx = (uint64_t)(t < 0 ? 0 : (t >= npx ? npx - 1 : t));
            } else {
                cx = (uint64_t)fx;
            }
            if (Ly > 0.0) {
                int64_t t = (int64_t)fy;
                cy = (uint64_t)(t < 0 ? 0 : (t >= npy ? npy - 1 : t));
            } else {
                cy = (uint64_t)fy;
            }
            if (cx >= (1u << 21) || cy >= (1u << 21) || cz >= (1u << 21)) bad = 1;
            t[i].key = spread3(cx) | (spread3(cy) << 1) | (spread3(cz) << 2);
            t[i].idx = i;
        }
        qsort(t + a, (size_t)(b - a), sizeof(KeyIdx), cmp_keyidx);
    }
    for (int64_t i = 0; i < n; ++i) {
        perm[i] = (int32_t)t[i].idx;
        if (keys) keys[i] = t[i].key;
    }
    free(t);
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Neighbour data: mirrors, candidates, stencils, ghosts.              */
/* ------------------------------------------------------------------ */

typedef struct {
    int64_t n, n_m, n_cand;
    int32_t n_sys;
    int64_t* off;
    double* prm;
    double cfg[C_NCFG];
    int32_t* sys;                 /* system of each real particle        */
    /* all points: reals 0..n-1 then mirrors n..n+n_m-1 */
    double *px, *py, *pz, *pu, *pv, *pw, *pV;
    int32_t* msrc;                /* source real of each mirror          */
    int64_t* coff;                /* candidates, CSR sorted by id        */
    int32_t* cidx;
    int32_t* scnt;                /* stencil count (without ghosts)      */
    int32_t* sidx;                /* n x m_max, canonical order          */
    uint8_t* gmask;               /* uncovered octants -> ghost rows     */
    int m_max;
} OrcNbr;

static int32_t point_sys(const OrcNbr* h, int64_t j)
{
    return j < h->n ? h->sys[j] : h->sys[h->msrc[j - h->n]];
}

/* displacement from real i to point j, through the nearest periodic image
 * of j along periodic axes */
static void disp(const OrcNbr* h, int64_t i, int64_t j, double* dx, double* dy,
                 double* dz)
{
    const double* p = h->prm + (size_t)h->sys[i] * P_NPRM;
    *dx = image_coord(h->px[j], h->px[i], p[P_LX]) - h->px[i];
    *dy = image_coord(h->py[j], h->py[i], p[P_LY]) - h->py[i];
    *dz = h->pz[j] - h->pz[i];
}

/* candidate test of Sec. 3.1 step 5: strict r2 < R2, r2 summed left to
 * right, no fused multiply-add (the file is built with contraction off) */
static int is_candidate(const OrcNbr* h, int64_t i, int64_t j, double R2,
                        double* r2o)
{
    double dx, dy, dz;
    disp(h, i, j, &dx, &dy, &dz);
    double r2 = dx * dx + dy * dy;
    r2 = r2 + dz * dz;
    *r2o = r2;
    return r2 < R2;
}

static int cmp_i32(const void* a, const void* b)
{
    int32_t p = *(const int32_t*)a, q = *(const int32_t*)b;
    return p < q ? -1 : (p > q);
}

/* Collects the candidate ids of real i, ascending.  brute: scan every
 * point of the system.  Otherwise a uniform bucket grid (edge 1.01 R, so
 * every point within R lies in the 27 surrounding buckets). */
typedef struct {
    double x0, y0, z0, ic, icx, icy;
    double xlo, ylo, Lx, Ly;  /* periodic box (L = 0: open axis) */
    int64_t nx, ny, nz;
    int64_t* start;   /* bucket start in items, size nx*ny*nz + 1 */
    int64_t* items;   /* point ids grouped by bucket             */
} Grid;

static int64_t grid_cell(const Grid* g, double x, double y, double z,
                         int64_t* cx, int64_t* cy, int64_t* cz)
{
    x = wrap_coord(x, g->xlo, g->Lx);
    y = wrap_coord(y, g->ylo, g->Ly);
    *cx = (int64_t)floor((x - g->x0) * g->icx);
    *cy = (int64_t)floor((y - g->y0) * g->icy);
    *cz = (int64_t)floor((z - g->z0) * g->ic);
    if (*cx < 0) *cx = 0;
    if (*cy < 0) *cy = 0;
    if (*cz < 0) *cz = 0;
    if (*cx >= g->nx) *cx = g->nx - 1;
    if (*cy >= g->ny) *cy = g->ny - 1;
    if (*cz >= g->nz) *cz = g->nz - 1;
    return *cx + g->nx * (*cy + g->ny * *cz);
}

static void build_grids(OrcNbr* h, Grid* grids)
{
    int64_t np = h->n + h->n_m;
    for (int s = 0; s < h->n_sys; ++s) {
        Grid* g = &grids[s];
        const double* p = h->prm + (size_t)s * P_NPRM;
        double lo[3] = {INFINITY, INFINITY, INFINITY};
        double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        int64_t cnt = 0;
        for (int64_t j = 0; j < np; ++j) {
            if (point_sys(h, j) != s) continue;
            double q[3] = {h->px[j], h->py[j], h->pz[j]};
            for (int a = 0; a < 3; ++a) {
                if (q[a] < lo[a]) lo[a] = q[a];
                if (q[a] > hi[a]) hi[a] = q[a];
            }
            ++cnt;
        }
        double edge = 1.01 * p[P_R];
        g->ic = g->icx = g->icy = 1.0 / edge;
        if (cnt == 0) { lo[0] = lo[1] = lo[2] = 0; hi[0] = hi[1] = hi[2] = 0; }
        g->x0 = lo[0]; g->y0 = lo[1]; g->z0 = lo[2];
        g->nx = (int64_t)floor((hi[0] - lo[0]) * g->ic) + 1;
        g->ny = (int64_t)floor((hi[1] - lo[1]) * g->ic) + 1;
        g->nz = (int64_t)floor((hi[2] - lo[2]) * g->ic) + 1;
        g->xlo = p[P_XLO]; g->ylo = p[P_YLO]; g->Lx = p[P_LX]; g->Ly = p[P_LY];
        if (g->Lx > 0.0) {
            g->x0 = g->xlo;
            g->nx = periodic_cells(g->Lx, g->ic);
            g->icx = (double)g->nx / g->Lx;
        }
        if (g->Ly > 0.0) {
            g->y0 = g->ylo;
            g->ny = periodic_cells(g->Ly, g->ic);
            g->icy = (double)g->ny / g->Ly;
        }
        int64_t nc = g->nx * g->ny * g->nz;
        g->start = (int64_t*)calloc((size_t)nc + 1, sizeof(int64_t));
        g->items = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cnt > 0 ? cnt : 1));
        int64_t cx, cy, cz;
        for (int64_t j = 0; j < np; ++j) {
            if (point_sys(h, j) != s) continue;
            g->start[grid_cell(g, h->px[j], h->py[j], h->pz[j], &cx, &cy, &cz) + 1]++;
        }
        for (int64_t c = 0; c < nc; ++c) g->start[c + 1] += g->start[c];
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nc + 1));
        memcpy(fill, g->start, sizeof(int64_t) * (size_t)(nc + 1));
        for (int64_t j = 0; j < np; ++j) {
            if (point_sys(h, j) != s) continue;
            int64_t c = grid_cell(g, h->px[j], h->py[j], h->pz[j], &cx, &cy, &cz);
            g->items[fill[c]++] = j;
        }
        free(fill);
    }
}

static int collect(const OrcNbr* h, const Grid* grids, int brute, int64_t i,
                   int32_t* out, int cap)
{
    int32_t s = h->sys[i];
    const double* p = h->prm + (size_t)s * P_NPRM;
    double R2 = p[P_R] * p[P_R];
    int cnt = 0;
    double r2;
    if (brute) {
        for (int64_t j = h->off[s]; j < h->off[s + 1]; ++j)
            if (j != i && is_candidate(h, i, j, R2, &r2)) {
                if (cnt < cap) out[cnt] = (int32_t)j;
                ++cnt;
            }
        for (int64_t k = 0; k < h->n_m; ++k) {
            int64_t j = h->n + k;
            if (h->sys[h->msrc[k]] == s && is_candidate(h, i, j, R2, &r2)) {
                if (cnt < cap) out[cnt] = (int32_t)j;
                ++cnt;
            }
        }
        return cnt;
    }
    const Grid* g = &grids[s];
    int64_t cx, cy, cz;
    grid_cell(g, h->px[i], h->py[i], h->pz[i], &cx, &cy, &cz);
    /* along a periodic axis the neighbouring cells wrap around; with fewer
     * than three cells each is visited once */
    for (int64_t z = cz - 1; z <= cz + 1; ++z)
        for (int64_t ya = cy - 1; ya <= cy + 1; ++ya)
            for (int64_t xa = cx - 1; xa <= cx + 1; ++xa) {
                int64_t x = xa, y = ya;
                if (g->Lx > 0.0) {
                    if (xa - cx >= g->nx || cx - xa >= g->nx) continue;
                    if (g->nx == 2 && xa == cx - 1) continue;
                    x = (xa % g->nx + g->nx) % g->nx;
                }
                if (g->Ly > 0.0) {
                    if (ya - cy >= g->ny || cy - ya >= g->ny) continue;
                    if (g->ny == 2 && ya == cy - 1) continue;
                    y = (ya % g->ny + g->ny) % g->ny;
                }
                if (x < 0 || y < 0 || z < 0 || x >= g->nx || y >= g->ny || z >= g->nz)
                    continue;
                int64_t c = x + g->nx * (y + g->ny * z);
                for (int64_t t = g->start[c]; t < g->start[c + 1]; ++t) {
                    int64_t j = g->items[t];
                    if (j != i && is_candidate(h, i, j, R2, &r2)) {
                        if (cnt < cap) out[cnt] = (int32_t)j;
                        ++cnt;
                    }
                }
            }
    if (cnt <= cap) qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);
    return cnt;
}

typedef struct { double r2; int32_t id; int oct; } Cand;

static int cmp_cand(const void* a, const void* b)
{
    const Cand* p = (const Cand*)a;
    const Cand* q = (const Cand*)b;
    if (p->r2 != q->r2) return p->r2 < q->r2 ? -1 : 1;
    return p->id < q->id ? -1 : (p->id > q->id);
}

/* Stencil of real i from its candidate list (Sec. 3.1 step 6): order by
 * key (r2, id); octant o = [dx>=0] + 2[dy>=0] + 4[dz>=0]; for o = 0..7
 * the first candidate with octant o, then every other candidate in key
 * order; truncate to m_max.  Ghost mask (Sec. 3.1 steps 5, 9): octant
 * s in {-1,1}^3 (bit [sx>0] + 2[sy>0] + 4[sz>0]) is covered iff some
 * candidate has s_a d_a > margin for every axis; uncovered octants get a
 * ghost. */
static void make_stencil(const OrcNbr* h, int64_t i, const int32_t* cand,
                         int nc, int32_t* sten, int* ns, uint8_t* gm)
{
    const double* p = h->prm + (size_t)h->sys[i] * P_NPRM;
    double margin = h->cfg[C_GMARGIN] * p[P_H];
    Cand* c = (Cand*)malloc(sizeof(Cand) * (size_t)(nc > 0 ? nc : 1));
    unsigned covered = 0;
    for (int t = 0; t < nc; ++t) {
        int64_t j = cand[t];
        double dx, dy, dz;
        disp(h, i, j, &dx, &dy, &dz);
        double r2 = dx * dx + dy * dy;
        r2 = r2 + dz * dz;
        c[t].r2 = r2;
        c[t].id = (int32_t)j;
        c[t].oct = (dx >= 0) + 2 * (dy >= 0) + 4 * (dz >= 0);
        for (int o = 0; o < 8; ++o) {
            double sx = (o & 1) ? 1.0 : -1.0, sy = (o & 2) ? 1.0 : -1.0,
                   sz = (o & 4) ? 1.0 : -1.0;
            if (sx * dx > margin && sy * dy > margin && sz * dz > margin)
                covered |= 1u << o;
        }
    }
    qsort(c, (size_t)nc, sizeof(Cand), cmp_cand);
    int taken_first[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    for (int o = 0; o < 8; ++o)
        for (int t = 0; t < nc; ++t)
            if (c[t].oct == o) { taken_first[o] = t; break; }
    int m = 0;
    for (int o = 0; o < 8; ++o)
        if (taken_first[o] >= 0 && m < h->m_max) sten[m++] = c[taken_first[o]].id;
    for (int t = 0; t < nc && m < h->m_max; ++t) {
        int first = 0;
        for (int o = 0; o < 8; ++o) if (taken_first[o] == t) first = 1;
        if (!first) sten[m++] = c[t].id;
    }
    *ns = m;
    *gm = (uint8_t)(~covered & 0xFFu);
    free(c);
}

void orc_nbr_free(void* hp)
{
    OrcNbr* h = (OrcNbr*)hp;
    if (!h) return;
    free(h->off); free(h->prm); free(h->sys);
    free(h->px); free(h->py); free(h->pz); free(h->pu); free(h->pv);
    free(h->pw); free(h->pV); free(h->msrc); free(h->coff); free(h->cidx);
    free(h->scnt); free(h->sidx); free(h->gmask);
    free(h);
}

/* Builds mirrors, candidate lists, stencils and ghost masks for the
 * particles in the order given.  Mirrors (Sec. 3.1 step 9): for each real
 * i, ascending, with z_i - wall < R, a mirror at (x, y, 2 wall - z) with
 * velocity (u, v, -w), the same V, id n + k. */
void* orc_nbr_build(int64_t n, int32_t n_sys, const int64_t* off,
                    const double* prm, const double* cfg,
                    const double* x, const double* y, const double* z,
                    const double* u, const double* v, const double* w,
                    const double* V, int brute)
{
    OrcNbr* h = (OrcNbr*)calloc(1, sizeof(OrcNbr));
    h->n = n;
    h->n_sys = n_sys;
    h->off = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_sys + 1));
    memcpy(h->off, off, sizeof(int64_t) * (size_t)(n_sys + 1));
    h->prm = (double*)malloc(sizeof(double) * (size_t)n_sys * P_NPRM);
    memcpy(h->prm, prm, sizeof(double) * (size_t)n_sys * P_NPRM);
    memcpy(h->cfg, cfg, sizeof(double) * C_NCFG);
    h->m_max = (int)cfg[C_MMAX];
    h->sys = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int s = 0; s < n_sys; ++s)
        for (int64_t i = off[s]; i < off[s + 1]; ++i) h->sys[i] = s;

    int64_t nm = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double* p = prm + (size_t)h->sys[i] * P_NPRM;
        if (z[i] - p[P_WALL] < p[P_R]) ++nm;
    }
    h->n_m = nm;
    int64_t np = n + nm;
    size_t sz = sizeof(double) * (size_t)(np > 0 ? np : 1);
    h->px = (double*)malloc(sz); h->py = (double*)malloc(sz);
    h->pz = (double*)malloc(sz); h->pu = (double*)malloc(sz);
    h->pv = (double*)malloc(sz); h->pw = (double*)malloc(sz);
    h->pV = (double*)malloc(sz);
    h->msrc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nm > 0 ? nm : 1));
    memcpy(h->px, x, sizeof(double) * (size_t)n);
    memcpy(h->py, y, sizeof(double) * (size_t)n);
    memcpy(h->pz, z, sizeof(double) * (size_t)n);
    memcpy(h->pu, u, sizeof(double) * (size_t)n);
    memcpy(h->pv, v, sizeof(double) * (size_t)n);
    memcpy(h->pw, w, sizeof(double) * (size_t)n);
    memcpy(h->pV, V, sizeof(double) * (size_t)n);
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        const double* p = prm + (size_t)h->sys[i] * P_NPRM;
        if (z[i] - p[P_WALL] < p[P_R]) {
            int64_t j = n + k;
            h->px[j] = x[i];
            h->py[j] = y[i];
            h->pz[j] = 2.0 * p[P_WALL] - z[i];
            h->pu[j] = u[i];
            h->pv[j] = v[i];
            h->pw[j] = -w[i];
            h->pV[j] = V[i];
            h->msrc[k] = (int32_t)i;
            ++k;
        }
    }

    Grid* grids = NULL;
    if (!brute) {
        grids = (Grid*)calloc((size_t)(n_sys > 0 ? n_sys : 1), sizeof(Grid));
        build_grids(h, grids);
    }
    /* pass 1: counts */
    int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int32_t tmp[1];
        cnt[i] = collect(h, grids, brute, i, tmp, 0);
    }
    h->coff = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    h->coff[0] = 0;
    for (int64_t i = 0; i < n; ++i) h->coff[i + 1] = h->coff[i] + cnt[i];
    h->n_cand = h->coff[n];
    h->cidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)(h->n_cand > 0 ? h->n_cand : 1));
    h->scnt = (int32_t*)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    h->sidx = (int32_t*)calloc((size_t)(n > 0 ? n : 1) * (size_t)h->m_max, sizeof(int32_t));
    h->gmask = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int nc = (int)cnt[i];
        collect(h, grids, brute, i, h->cidx + h->coff[i], nc);
        int ns = 0;
        make_stencil(h, i, h->cidx + h->coff[i], nc,
                     h->sidx + (size_t)i * h->m_max, &ns, &h->gmask[i]);
        h->scnt[i] = ns;
    }
    free(cnt);
    if (grids) {
        for (int s = 0; s < n_sys; ++s) { free(grids[s].start); free(grids[s].items); }
        free(grids);
    }
    return h;
}

void orc_nbr_sizes(void* hp, int64_t* out)
{
    OrcNbr* h = (OrcNbr*)hp;
    out[0] = h->n_m;
    out[1] = h->n_cand;
    out[2] = h->m_max;
}

void orc_nbr_export(void* hp, int64_t* coff, int32_t* cidx, int32_t* scnt,
                    int32_t* sidx, uint8_t* gmask, int32_t* msrc,
                    double* mirror7 /* 7 x n_m: x y z u v w V */)
{
    OrcNbr* h = (OrcNbr*)hp;
    int64_t n = h->n, nm = h->n_m;
    if (coff) memcpy(coff, h->coff, sizeof(int64_t) * (size_t)(n + 1));
    if (cidx) memcpy(cidx, h->cidx, sizeof(int32_t) * (size_t)h->n_cand);
    if (scnt) memcpy(scnt, h->scnt, sizeof(int32_t) * (size_t)n);
    if (sidx) memcpy(sidx, h->sidx, sizeof(int32_t) * (size_t)n * (size_t)h->m_max);
    if (gmask) memcpy(gmask, h->gmask, (size_t)n);
    if (msrc) memcpy(msrc, h->msrc, sizeof(int32_t) * (size_t)nm);
    if (mirror7) {
        const double* src[7] = {h->px, h->py, h->pz, h->pu, h->pv, h->pw, h->pV};
        for (int a = 0; a < 7; ++a)
            memcpy(mirror7 + (size_t)a * nm, src[a] + n, sizeof(double) * (size_t)nm);
    }
}

/* ------------------------------------------------------------------ */
/* Least squares by Householder QR.                                    */
/* ------------------------------------------------------------------ */

/* min || A c - B ||_2 for the m x nc matrix A (row-major, leading dim lda)
 * and nb right-hand sides B (row-major, leading dim ldb).  Householder QR
 * without pivoting (Golub & Van Loan, Matrix Computations, Householder QR
 * and its least-squares use): for each column j the reflector
 * I - 2 v v^T / (v^T v) with v = x - alpha e_1, alpha = -sign(x_1) ||x||,
 * is applied to the remaining columns and to B; then R c = (Q^T B)[0:nc]
 * is solved by back substitution.  A and B are overwritten.  Returns
 * min_j |r_jj| / max_j |r_jj| (0 when a column vanishes).  Requires
 * m >= nc. */
static double house_lsq(int m, int nc, double* A, int lda, double* B,
                        int ldb, int nb, double* C /* nc x nb, ld nb */)
{
    double rd[NC3];
    double rmin = INFINITY, rmax = 0.0;
    for (int j = 0; j < nc; ++j) {
        double s = 0.0;
        for (int r = j; r < m; ++r) s += A[r * lda + j] * A[r * lda + j];
        double nrm = sqrt(s);
        double ajj = A[j * lda + j];
        if (nrm == 0.0) {
            rd[j] = 0.0;
            rmin = 0.0;
            continue;
        }
        double alpha = ajj >= 0.0 ? -nrm : nrm;
        A[j * lda + j] = ajj - alpha;
        double vtv = 2.0 * nrm * (nrm + fabs(ajj));
        for (int l = j + 1; l < nc; ++l) {
            double dot = 0.0;
            for (int r = j; r < m; ++r) dot += A[r * lda + j] * A[r * lda + l];
            double f = 2.0 * dot / vtv;
            for (int r = j; r < m; ++r) A[r * lda + l] -= f * A[r * lda + j];
        }
        for (int l = 0; l < nb; ++l) {
            double dot = 0.0;
            for (int r = j; r < m; ++r) dot += A[r * lda + j] * B[r * ldb + l];
            double f = 2.0 * dot / vtv;
            for (int r = j; r < m; ++r) B[r * ldb + l] -= f * A[r * lda + j];
        }
        rd[j] = alpha;
        double ar = fabs(alpha);
        if (ar < rmin) rmin = ar;
        if (ar > rmax) rmax = ar;
    }
    for (int l = 0; l < nb; ++l)
        for (int j = nc - 1; j >= 0; --j) {
            double acc = B[j * ldb + l];
            for (int q = j + 1; q < nc; ++q) acc -= A[j * lda + q] * C[q * nb + l];
            C[j * nb + l] = rd[j] != 0.0 ? acc / rd[j] : 0.0;
        }
    return rmax > 0.0 ? rmin / rmax : 0.0;
}

/* Taylor row of Sec. 3.1 step 7 in 3D, scaled by h:
 * (xi_x, xi_y, xi_z, xi_x^2/2, xi_y^2/2, xi_z^2/2, xi_x xi_y, xi_x xi_z,
 *  xi_y xi_z) with xi = (x_k - x_i) / h. */
static void taylor_row(double ex, double ey, double ez, double* a)
{
    a[0] = ex; a[1] = ey; a[2] = ez;
    a[3] = 0.5 * ex * ex; a[4] = 0.5 * ey * ey; a[5] = 0.5 * ez * ez;
    a[6] = ex * ey; a[7] = ex * ez; a[8] = ey * ez;
}

/* Third-order Taylor row (the higher-order fit the paper lists as further
 * work): the quadratic row followed by the cubic monomials divided by the
 * factorials of their exponents, so that each coefficient is the matching
 * third derivative times h^3:
 * xi_x^3/6, xi_y^3/6, xi_z^3/6, xi_x^2 xi_y/2, xi_x^2 xi_z/2,
 * xi_y^2 xi_x/2, xi_y^2 xi_z/2, xi_z^2 xi_x/2, xi_z^2 xi_y/2,
 * xi_x xi_y xi_z. */
static void taylor_row3(double ex, double ey, double ez, double* a)
{
    taylor_row(ex, ey, ez, a);
    a[9] = ex * ex * ex / 6.0; a[10] = ey * ey * ey / 6.0; a[11] = ez * ez * ez / 6.0;
    a[12] = 0.5 * ex * ex * ey; a[13] = 0.5 * ex * ex * ez;
    a[14] = 0.5 * ey * ey * ex; a[15] = 0.5 * ey * ey * ez;
    a[16] = 0.5 * ez * ez * ex; a[17] = 0.5 * ez * ez * ey;
    a[18] = ex * ey * ez;
}

#define FLAG_LINEAR 1u
#define FLAG_QUAD 16u

/* Fits nf fields at real i on its stencil plus ghost rows.
 * val(j, f): value of field f at point j (real or mirror).
 * gval[f]: value at the ghosts of i.  Output coef[f*9 + c]: derivative
 * estimates d_x, d_y, d_z, d_xx, d_yy, d_zz, d_xy, d_xz, d_yz.
 * Weights: unit (cfg weight 0) or exp(-4 r^2 / R^2) (cfg weight 1).
 * Fallback (reading of the paper, which is silent on degenerate
 * stencils): fewer than 9 rows, or min|r_jj|/max|r_jj| below the
 * configured tolerance, gives a 3-column linear fit with zero second
 * derivatives and sets FLAG_LINEAR.  With fit_order 3 the fit has the 19
 * columns of taylor_row3 and falls back the same way to the quadratic fit
 * (fewer than 19 rows or the ratio test; FLAG_QUAD), then to the linear
 * one.  Only the first and second derivatives are returned. */
typedef double (*field_fn)(const void* ctx, int64_t j, int f);

static unsigned fit_point(const OrcNbr* h, int64_t i, int nf, field_fn val,
                          const void* fctx, const double* gval, double* coef)
{
    const double* p = h->prm + (size_t)h->sys[i] * P_NPRM;
    double hh = p[P_H], R2 = p[P_R] * p[P_R];
    int ns = h->scnt[i];
    const int32_t* st = h->sidx + (size_t)i * h->m_max;
    uint8_t gm = h->gmask[i];
    int m = ns;
    for (int o = 0; o < 8; ++o) if (gm & (1u << o)) ++m;
    double A[MAXROWS * NC3], A2[MAXROWS * NC3];
    double B[MAXROWS * 8], B2[MAXROWS * 8], C[NC3 * 8];
    const int nc = h->cfg[C_ORDER] == 3.0 ? NC3 : NC;
    double fi[8];
    for (int f = 0; f < nf; ++f) fi[f] = val(fctx, i, f);
    int r = 0;
    for (int t = 0; t < ns; ++t, ++r) {
        int64_t j = st[t];
        double dx, dy, dz;
        disp(h, i, j, &dx, &dy, &dz);
        double wt = 1.0;
        if (h->cfg[C_WEIGHT] == 1.0) {
            double r2 = dx * dx + dy * dy + dz * dz;
            wt = sqrt(exp(-4.0 * r2 / R2));
        }
        taylor_row3(dx / hh, dy / hh, dz / hh, A + r * NC3);
        for (int c = 0; c < NC3; ++c) A[r * NC3 + c] *= wt;
        for (int f = 0; f < nf; ++f) B[r * 8 + f] = wt * (val(fctx, j, f) - fi[f]);
    }
    for (int o = 0; o < 8; ++o) {
        if (!(gm & (1u << o))) continue;
        double sx = (o & 1) ? 1.0 : -1.0, sy = (o & 2) ? 1.0 : -1.0,
               sz = (o & 4) ? 1.0 : -1.0;
        double wt = 1.0;
        if (h->cfg[C_WEIGHT] == 1.0) wt = sqrt(exp(-4.0 * 3.0 * hh * hh / R2));
        taylor_row3(sx, sy, sz, A + r * NC3);
        for (int c = 0; c < NC3; ++c) A[r * NC3 + c] *= wt;
        for (int f = 0; f < nf; ++f) B[r * 8 + f] = wt * (gval[f] - fi[f]);
        ++r;
    }
    unsigned flags = 0;
    double ratio = 0.0;
    int ok = 0;
    for (int f = 0; f < nf * NC3; ++f) C[f] = 0.0;
    /* a stencil with fewer real (or mirror) rows than min_real_rows takes
     * the linear fit whatever its ghost rows add (a reading: with as many
     * ghost rows as real ones the higher-order fit interpolates) */
    const int enough_real = ns >= h->cfg[C_MINREAL];
    if (nc == NC3 && m >= NC3 && enough_real) {
        memcpy(A2, A, sizeof(double) * (size_t)m * NC3);
        memcpy(B2, B, sizeof(double) * (size_t)m * 8);
        ratio = house_lsq(m, NC3, A2, NC3, B2, 8, nf, C);
        ok = ratio >= h->cfg[C_FTOL];
    }
    if (!ok) {
        if (nc == NC3) flags |= FLAG_QUAD;
        ratio = 0.0;
        if (m >= NC && enough_real) {
            memcpy(A2, A, sizeof(double) * (size_t)m * NC3);
            memcpy(B2, B, sizeof(double) * (size_t)m * 8);
            ratio = house_lsq(m, NC, A2, NC3, B2, 8, nf, C);
        }
        if (m < NC || !enough_real || ratio < h->cfg[C_FTOL]) {
            flags |= FLAG_LINEAR;
            for (int f = 0; f < nf * NC3; ++f) C[f] = 0.0;
            if (m >= 3) {
                double C3[3 * 8];
                memcpy(A2, A, sizeof(double) * (size_t)m * NC3);
                memcpy(B2, B, sizeof(double) * (size_t)m * 8);
                house_lsq(m, 3, A2, NC3, B2, 8, nf, C3);
                for (int c = 0; c < 3; ++c)
                    for (int f = 0; f < nf; ++f) C[c * nf + f] = C3[c * nf + f];
            }
        }
    }
    for (int f = 0; f < nf; ++f)
        for (int c = 0; c < NC; ++c)
            coef[f * NC + c] = C[c * nf + f] / (c < 3 ? hh : hh * hh);
    return flags;
}

/* ---- generic field fit (lp_fit_derivs parity) ---- */
typedef struct {
    const OrcNbr* h;
    const double* f;          /* nf x n values at reals */
    const int32_t* msign;     /* mirror value = msign[f] * value at source */
} GenCtx;

static double gen_val(const void* c, int64_t j, int f)
{
    const GenCtx* g = (const GenCtx*)c;
    int64_t n = g->h->n;
    if (j < n) return g->f[(size_t)f * n + j];
    return (double)g->msign[f] * g->f[(size_t)f * n + g->h->msrc[j - n]];
}

/* Fits nf (<= 8) fields given at the reals.  Mirror value = msign[f] times
 * the value at the mirror's source; ghost value = the particle's own value
 * (gzero[f] == 0) or zero (gzero[f] == 1).  coef is nf x 9 x n. */
int orc_fit(void* hp, const double* f, int nf, const int32_t* msign,
            const int32_t* gzero, double* coef, uint8_t* flags)
{
    OrcNbr* h = (OrcNbr*)hp;
    if (nf < 1 || nf > 8) return -1;
    GenCtx g = {h, f, msign};
    int64_t n = h->n;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double gv[8], c[8 * NC];
        for (int q = 0; q < nf; ++q) gv[q] = gzero[q] ? 0.0 : f[(size_t)q * n + i];
        unsigned fl = fit_point(h, i, nf, gen_val, &g, gv, c);
        for (int q = 0; q < nf; ++q)
            for (int k = 0; k < NC; ++k)
                coef[((size_t)q * NC + k) * n + i] = c[q * NC + k];
        if (flags) flags[i] = (uint8_t)fl;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* mu(I) closure (Sec. 2.2 and 2.2.1).                                  */
/* ------------------------------------------------------------------ */

enum { BR_GAS = 0, BR_INERTIAL = 1, BR_QUASI = 2 };

/* From the velocity gradient G[a][b] = d u_a / d x_b and the specific
 * volume V: strain rate D = (G + G^T)/2, shear rate gd = D - div/3 I,
 * |gd| = sqrt(gd:gd / 2), phi = 1/V, and the pressure law EOS2 with the
 * shear stress of eqs. friction/align:
 *   gas       phi <= phi_min:            P = 0, eta = 0
 *   inertial  phi_min < phi <= phi_max:  P = rho_s (2 a d |gd| / (phi_c - phi))^2,
 *             I = (phi_c - phi)/a (eq. inertialdensity, equal to eq.
 *             inertial for this P), mu(I) = mu_s + (mu_2 - mu_s)/(I0/I + 1),
 *             eta = mu P / |gd| = rho_s mu (2 a d / (phi_c - phi))^2 |gd|
 *   quasi-static phi > phi_max:          P = rho_s (alpha + beta phi), eta = 0
 * with a = phi_c - phi_min.  I and mu are reported as 0 outside the
 * inertial branch. */
static int closure(const double* p, double V, const double G[3][3],
                   double gd[3][3], double* out5 /* P eta I mu |gd| */)
{
    double div = G[0][0] + G[1][1] + G[2][2];
    double ss = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double D = 0.5 * (G[a][b] + G[b][a]);
            gd[a][b] = D - (a == b ? div / 3.0 : 0.0);
            ss += gd[a][b] * gd[a][b];
        }
    double gn = sqrt(0.5 * ss);
    double phi = 1.0 / V;
    double P = 0.0, eta = 0.0, I = 0.0, mu = 0.0;
    int br;
    if (phi <= p[P_PHIMIN]) {
        br = BR_GAS;
    } else if (phi <= p[P_PHIMAX]) {
        br = BR_INERTIAL;
        double a = p[P_PHIC] - p[P_PHIMIN];
        double wd = p[P_PHIC] - phi;
        double k = 2.0 * a * p[P_D] / wd;
        P = p[P_RHO] * (k * gn) * (k * gn);
        I = wd / a;
        mu = p[P_MUS] + (p[P_MU2] - p[P_MUS]) / (p[P_I0] / I + 1.0);
        eta = p[P_RHO] * mu * k * k * gn;
    } else {
        br = BR_QUASI;
        P = p[P_RHO] * (p[P_ALPHA] + p[P_BETA] * phi);
    }
    out5[0] = P; out5[1] = eta; out5[2] = I; out5[3] = mu; out5[4] = gn;
    return br;
}

/* pressure at a mirror particle: the source's density with zero shear
 * rate (Sec. 3.1 step 9, mirror particles) */
static double mirror_pressure(const double* p, double V)
{
    double phi = 1.0 / V;
    if (phi > p[P_PHIMAX]) return p[P_RHO] * (p[P_ALPHA] + p[P_BETA] * phi);
    return 0.0;
}

/* ---- full right-hand side ---- */
typedef struct {
    const OrcNbr* h;
    const double* P;
    const double* eta;
} P2Ctx;

static double vel_val(const void* c, int64_t j, int f)
{
    const OrcNbr* h = (const OrcNbr*)c;
    return f == 0 ? h->pu[j] : (f == 1 ? h->pv[j] : h->pw[j]);
}

static double p2_val(const void* c, int64_t j, int f)
{
    const P2Ctx* q = (const P2Ctx*)c;
    int64_t n = q->h->n;
    if (j < n) return f == 0 ? q->P[j] : q->eta[j];
    if (f == 1) return 0.0;
    int64_t s = q->h->msrc[j - n];
    const double* p = q->h->prm + (size_t)q->h->sys[s] * P_NPRM;
    double Pm = mirror_pressure(p, q->h->pV[j]);
    /* hydrostatic wall pressure (an option, after Adami, Hu & Adams 2012):
     * the mirror also carries the weight of the layer between it and its
     * source, rho_s phi_src |g_z| (z_src - z_mirror) */
    if (q->h->cfg[C_WALLP] == 1.0)
        Pm = Pm + p[P_RHO] * (1.0 / q->h->pV[j]) * (-p[P_GZ]) * (q->h->pz[s] - q->h->pz[j]);
    return Pm;
}

static const int HIDX[3][3] = {{3, 6, 7}, {6, 4, 8}, {7, 8, 5}};

/* Form M data (oracle cross-check only) */
typedef struct {
    const OrcNbr* h;
    const double* gn;
} MCtx;

static double m_val(const void* c, int64_t j, int f)
{
    const MCtx* q = (const MCtx*)c;
    int64_t n = q->h->n;
    if (f == 0) return q->h->pV[j];
    return j < n ? q->gn[j] : 0.0;
}

/* Evaluates the RHS for every real particle (Form E):
 *   pass 1: fit u, v, w  -> G (gradient), H (second derivatives)
 *   closure             -> P, eta (and I, mu, |gd|)
 *   pass 2: fit P, eta   -> grad P, grad eta
 *   a_a = V (-d_a P + gd_ab d_b eta + eta (Lap u_a / 2 + d_a div u / 6))
 *         / rho_s + g_a                               (eqs. sys2-sys4)
 *   dV/dt = V div u                                   (mass equation in V)
 * Outputs (each optional): coef_u 27 x n, diag 5 x n (P eta I mu |gd|),
 * grad 6 x n (dP/dx..z, deta/dx..z), acc 3 x n, dVdt n, flags n
 * (bit0 linear fallback, bits 1-2 branch).  accM 3 x n receives the
 * Form M acceleration (NaN where the particle is not inertial). */
int orc_eval(void* hp, double* coef_u, double* diag, double* grad,
             double* acc, double* dVdt, uint8_t* flags, double* accM)
{
    OrcNbr* h = (OrcNbr*)hp;
    int64_t n = h->n;
    double* P = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* eta = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* cu = (double*)malloc(sizeof(double) * 27 * (size_t)(n > 0 ? n : 1));
    double* gnv = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    uint8_t* fl = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const double* p = h->prm + (size_t)h->sys[i] * P_NPRM;
        double gv[3] = {h->pu[i], h->pv[i], h->pw[i]};
        double c[27];
        unsigned f1 = fit_point(h, i, 3, vel_val, h, gv, c);
        memcpy(cu + 27 * (size_t)i, c, sizeof(c));
        double G[3][3], gd[3][3], d5[5];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) G[a][b] = c[a * NC + b];
        int br = closure(p, h->pV[i], G, gd, d5);
        P[i] = d5[0];
        eta[i] = d5[1];
        gnv[i] = d5[4];
        fl[i] = (uint8_t)(f1 | (unsigned)(br << 1));
        if (diag)
            for (int q = 0; q < 5; ++q) diag[(size_t)q * n + i] = d5[q];
        if (coef_u)
            for (int q = 0; q < 27; ++q) coef_u[(size_t)q * n + i] = c[q];
    }
    P2Ctx pc = {h, P, eta};
    MCtx mc = {h, gnv};
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        const double* p = h->prm + (size_t)h->sys[i] * P_NPRM;
        double gv[2] = {0.0, 0.0};
        double c[18];
        fit_point(h, i, 2, p2_val, &pc, gv, c);
        const double* cq = cu + 27 * (size_t)i;
        double G[3][3], gd[3][3], d5[5];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) G[a][b] = cq[a * NC + b];
        closure(p, h->pV[i], G, gd, d5);
        double div = G[0][0] + G[1][1] + G[2][2];
        double V = h->pV[i];
        double gP[3] = {c[0], c[1], c[2]};
        double gE[3] = {c[NC + 0], c[NC + 1], c[NC + 2]};
        double e = eta[i];
        for (int a = 0; a < 3; ++a) {
            double lap = 0.0, gdiv = 0.0, tg = 0.0;
            for (int b = 0; b < 3; ++b) {
                lap += cq[a * NC + HIDX[b][b]];
                gdiv += cq[b * NC + HIDX[a][b]];
                tg += gd[a][b] * gE[b];
            }
            double force = -gP[a] + tg + e * (0.5 * lap + gdiv / 6.0);
            if (acc) acc[(size_t)a * n + i] = V * force / p[P_RHO] + p[P_GX + a];
        }
        if (dVdt) dVdt[i] = V * div;
        if (grad)
            for (int a = 0; a < 3; ++a) {
                grad[(size_t)a * n + i] = gP[a];
                grad[(size_t)(3 + a) * n + i] = gE[a];
            }
        if (accM) {
            int br = (fl[i] >> 1) & 3;
            if (br != BR_INERTIAL) {
                for (int a = 0; a < 3; ++a) accM[(size_t)a * n + i] = NAN;
            } else {
                /* ghost states for Form M: phi_G = frac * phi_min and
                 * |gd|_G = |gd|_i (phi_c - phi_G)/(phi_c - phi_i) */
                double phi = 1.0 / V;
                double phiG = h->cfg[C_PHIG] * p[P_PHIMIN];
                double gvm[2] = {1.0 / phiG,
                                 d5[4] * (p[P_PHIC] - phiG) / (p[P_PHIC] - phi)};
                double cm[18];
                fit_point(h, i, 2, m_val, &mc, gvm, cm);
                double aa = p[P_PHIC] - p[P_PHIMIN];
                double wd = p[P_PHIC] - phi;
                double dd = p[P_D];
                double M = -4.0 * aa * aa * dd * dd / (wd * wd);
                double mu = (aa * p[P_MUS] * p[P_I0] + p[P_MU2] * wd) / (aa * p[P_I0] + wd);
                double N = -M * mu;
                double S = -8.0 * aa * aa * dd * dd / (wd * wd * wd);
                double Rr = -S * mu + M * aa * p[P_I0] * (p[P_MU2] - p[P_MUS]) /
                            ((aa * p[P_I0] + wd) * (aa * p[P_I0] + wd));
                double gn = d5[4];
                for (int a = 0; a < 3; ++a) {
                    double lap = 0.0, gdiv = 0.0, t1 = 0.0, t2 = 0.0;
                    for (int b = 0; b < 3; ++b) {
                        lap += cq[a * NC + HIDX[b][b]];
                        gdiv += cq[b * NC + HIDX[a][b]];
                        t1 += gd[a][b] * cm[b];
                        t2 += gd[a][b] * cm[NC + b];
                    }
                    /* -R|gd|/V^2 ((S/R)|gd| V_a + gd_ab V_b) */
                    double term1 = -(S * gn * gn * cm[a] + Rr * gn * t1) / (V * V);
                    /* N ((2M/N)|gd| |gd|_a + gd_ab |gd|_b) */
                    double term2 = 2.0 * M * gn * cm[NC + a] + N * t2;
                    double term3 = N * gn * (0.5 * lap + gdiv / 6.0);
                    accM[(size_t)a * n + i] = V * (term1 + term2 + term3) + p[P_GX + a];
                }
            }
        }
    }
    if (flags) memcpy(flags, fl, (size_t)n);
    free(P); free(eta); free(cu); free(gnv); free(fl);
    return 0;
}

/* Explicit update (Sec. 3.1 step 8 and step 10):
 *   V' = V + dt dV/dt,  u' = u + dt a,  x' = x + dt (u + u') / 2.
 * Returns the number of particles that end below their wall plane. */
/* Reflecting wall (an option; the paper states only the mirror boundary):
 * a particle that ends a step below the wall plane is reflected across it,
 * z -> 2 wall - z, w -> -w. */
static void reflect_wall(double wall, double* z, double* w)
{
    if (*z < wall) {
        *z = 2.0 * wall - *z;
        *w = -*w;
    }
}

int64_t orc_update(int64_t n, int32_t n_sys, const int64_t* off,
                   const double* prm, double dt, double* x, double* y,
                   double* z, double* u, double* v, double* w, double* V,
                   const double* acc, const double* dVdt, int reflect)
{
    int64_t below = 0;
    for (int s = 0; s < n_sys; ++s) {
        const double* p = prm + (size_t)s * P_NPRM;
        for (int64_t i = off[s]; i < off[s + 1]; ++i) {
            double un = u[i] + dt * acc[i];
            double vn = v[i] + dt * acc[n + i];
            double wn = w[i] + dt * acc[2 * n + i];
            x[i] = wrap_coord(x[i] + dt * (0.5 * (u[i] + un)), p[P_XLO], p[P_LX]);
            y[i] = wrap_coord(y[i] + dt * (0.5 * (v[i] + vn)), p[P_YLO], p[P_LY]);
            z[i] = z[i] + dt * (0.5 * (w[i] + wn));
            u[i] = un; v[i] = vn; w[i] = wn;
            V[i] = V[i] + dt * dVdt[i];
            if (reflect) reflect_wall(p[P_WALL], &z[i], &w[i]);
            if (z[i] < p[P_WALL]) ++below;
        }
    }
    return below;
}

/* Boundary treatment of a step's result (used by the second-order step's
 * corrector): positions wrapped along the periodic axes into their box,
 * and with `reflect` the reflecting wall. */
void orc_boundary(int64_t n, int32_t n_sys, const int64_t* off, const double* prm,
                  double* x, double* y, double* z, double* w, int reflect)
{
    for (int s = 0; s < n_sys; ++s) {
        const double* p = prm + (size_t)s * P_NPRM;
        for (int64_t i = off[s]; i < off[s + 1]; ++i) {
            x[i] = wrap_coord(x[i], p[P_XLO], p[P_LX]);
            y[i] = wrap_coord(y[i], p[P_YLO], p[P_LY]);
            if (reflect) reflect_wall(p[P_WALL], &z[i], &w[i]);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Direct entry points used by the oracle's own pin tests.             */
/* ------------------------------------------------------------------ */

/* Raw least squares: A is m x nc (row-major), B is m x nb (row-major);
 * C receives nc x nb.  Inputs are copied.  Returns min|r_jj|/max|r_jj|. */
double orc_lsq(int m, int nc, const double* A, const double* B, int nb,
               double* Cout)
{
    if (m < nc || nc > NC3 || nb > 8 || m > MAXROWS) return -1.0;
    double A2[MAXROWS * NC3], B2[MAXROWS * 8];
    for (int r = 0; r < m; ++r) {
        for (int c = 0; c < nc; ++c) A2[r * NC3 + c] = A[r * nc + c];
        for (int l = 0; l < nb; ++l) B2[r * 8 + l] = B[r * nb + l];
    }
    return house_lsq(m, nc, A2, NC3, B2, 8, nb, Cout);
}

/* Closure at one point: G9 row-major d u_a / d x_b; out5 = P eta I mu |gd|;
 * gd9 receives the shear-rate tensor.  Returns the branch. */
int orc_closure_point(const double* prm, double V, const double* G9,
                      double* out5, double* gd9)
{
    double G[3][3], gd[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[a][b] = G9[3 * a + b];
    int br = closure(prm, V, G, gd, out5);
    if (gd9)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) gd9[3 * a + b] = gd[a][b];
    return br;
}
