// Device building blocks of the least-squares fits and the closure,
// shared by the step kernels and the adjoint kernels: Taylor rows
// (Sec. 3.1 step 7, 3D second order), Gram moments and Cholesky solves,
// the mu(I) closure (Sec. 2.2, 2.2.1), the viscous terms of the Form E
// right-hand side (Sec. 2.1) and the walk over a particle's fit rows.
#pragma once

#include "lp_visit.h"

namespace lp {

// upper-triangle index of (i, j), i <= j, in a packed 9x9
__host__ __device__ constexpr int uix(int i, int j)
{
    return i * 9 - (i * (i - 1)) / 2 + (j - i);
}

__device__ __forceinline__ void taylor_row(double ex, double ey, double ez,
                                           double a[9])
{
    a[0] = ex;
    a[1] = ey;
    a[2] = ez;
    a[3] = 0.5 * ex * ex;
    a[4] = 0.5 * ey * ey;
    a[5] = 0.5 * ez * ez;
    a[6] = ex * ey;
    a[7] = ex * ez;
    a[8] = ey * ez;
}

__device__ __forceinline__ void ghost_offset(int o, double& sx, double& sy,
                                             double& sz)
{
    sx = (o & 1) ? 1.0 : -1.0;
    sy = (o & 2) ? 1.0 : -1.0;
    sz = (o & 4) ? 1.0 : -1.0;
}

// Taylor row of a stencil point and its weight.
__device__ __forceinline__ double point_row(const View& v, const GridInfo& g,
                                            double dx, double dy, double dz,
                                            double a[9])
{
    taylor_row(dx * g.inv_h, dy * g.inv_h, dz * g.inv_h, a);
    if (v.weight == LP_W_GAUSS)
        return exp(-4.0 * (dx * dx + dy * dy + dz * dz) / g.R2);
    return 1.0;
}

// Taylor row of the ghost in octant o (offset h s) and its weight.
__device__ __forceinline__ double ghost_row(const View& v, const GridInfo& g, int o,
                                            double a[9])
{
    double sx, sy, sz;
    ghost_offset(o, sx, sy, sz);
    taylor_row(sx, sy, sz, a);
    if (v.weight == LP_W_GAUSS) return exp(-12.0 * g.h * g.h / g.R2);
    return 1.0;
}

// Velocity carried by a stencil point (mirrors reverse w).
__device__ __forceinline__ void point_velocity(const View& v, const Pt& p,
                                               double& u, double& vv, double& w)
{
    u = v.u[p.src];
    vv = v.v[p.src];
    w = p.mirror ? -v.w[p.src] : v.w[p.src];
}

// G = U^T U in place (packed upper, with 1 / U_jj stored on the diagonal
// for chol_solve); returns min U_jj / max U_jj, or -1 when a pivot is not
// positive.
template <int N, class T>
__device__ __forceinline__ T cholesky(T (&G)[45])
{
    T dmin = INFINITY, dmax = 0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T s = G[uix(j, j)];
#pragma unroll
        for (int k = 0; k < j; ++k) s -= G[uix(k, j)] * G[uix(k, j)];
        if (!(s > T(0))) return T(-1);
        const T d = sqrt(s);
        const T inv = T(1) / d;
        G[uix(j, j)] = inv;   // the solves multiply by the reciprocal pivot
        dmin = fmin(dmin, d);
        dmax = fmax(dmax, d);
#pragma unroll
        for (int l = j + 1; l < N; ++l) {
            T t = G[uix(j, l)];
#pragma unroll
            for (int k = 0; k < j; ++k) t -= G[uix(k, j)] * G[uix(k, l)];
            G[uix(j, l)] = t * inv;
        }
    }
    return dmin / dmax;
}

// Solves U^T U c = b in place (b -> c); U as cholesky leaves it (reciprocal
// pivots on the diagonal).
template <int N, class T>
__device__ __forceinline__ void chol_solve(const T (&U)[45], T (&b)[9])
{
#pragma unroll
    for (int j = 0; j < N; ++j) {
        T t = b[j];
#pragma unroll
        for (int k = 0; k < j; ++k) t -= U[uix(k, j)] * b[k];
        b[j] = t * U[uix(j, j)];
    }
#pragma unroll
    for (int j = N - 1; j >= 0; --j) {
        T t = b[j];
#pragma unroll
        for (int k = j + 1; k < N; ++k) t -= U[uix(j, k)] * b[k];
        b[j] = t * U[uix(j, j)];
    }
}

// ---- closure (Sec. 2.2 and 2.2.1) --------------------------------------

struct Closure {
    double gd[6];       // xx yy zz xy xz yz of the shear-rate tensor
    double div, gn, P, eta, I, mu;
    int branch;         // 0 gas, 1 inertial, 2 quasi-static
};

// c[f*9 + q]: derivative q of velocity component f.
__device__ __forceinline__ Closure closure(const lp_params& p, double V,
                                           const double (&c)[27])
{
    Closure r;
    const double gxx = c[0], gyy = c[9 + 1], gzz = c[18 + 2];
    r.div = gxx + gyy + gzz;
    const double third = r.div / 3.0;
    r.gd[0] = gxx - third;
    r.gd[1] = gyy - third;
    r.gd[2] = gzz - third;
    r.gd[3] = 0.5 * (c[1] + c[9 + 0]);      // (du/dy + dv/dx)/2
    r.gd[4] = 0.5 * (c[2] + c[18 + 0]);     // (du/dz + dw/dx)/2
    r.gd[5] = 0.5 * (c[9 + 2] + c[18 + 1]); // (dv/dz + dw/dy)/2
    const double ss = r.gd[0] * r.gd[0] + r.gd[1] * r.gd[1] + r.gd[2] * r.gd[2] +
                      2.0 * (r.gd[3] * r.gd[3] + r.gd[4] * r.gd[4] + r.gd[5] * r.gd[5]);
    r.gn = sqrt(0.5 * ss);
    const double phi = 1.0 / V;
    r.P = r.eta = r.I = r.mu = 0.0;
    if (phi <= p.phi_min) {
        r.branch = 0;
    } else if (phi <= p.phi_max) {
        r.branch = 1;
        const double a = p.phi_c - p.phi_min;
        const double w = p.phi_c - phi;
        const double k = 2.0 * a * p.d / w;
        r.P = p.rho_s * (k * r.gn) * (k * r.gn);
        r.I = w / a;
        r.mu = p.mu_s + (p.mu_2 - p.mu_s) / (p.I0 / r.I + 1.0);
        r.eta = p.rho_s * r.mu * k * k * r.gn;
    } else {
        r.branch = 2;
        r.P = p.rho_s * (p.alpha + p.beta * phi);
    }
    return r;
}

__device__ __forceinline__ double mirror_pressure(const lp_params& p, double V)
{
    const double phi = 1.0 / V;
    return phi > p.phi_max ? p.rho_s * (p.alpha + p.beta * phi) : 0.0;
}

// Lap u_a / 2 + d_a div u / 6 from the velocity coefficients.
__device__ __forceinline__ void visc_terms(const double (&c)[27], double (&vis)[3])
{
    const double lap0 = c[3] + c[4] + c[5];
    const double lap1 = c[9 + 3] + c[9 + 4] + c[9 + 5];
    const double lap2 = c[18 + 3] + c[18 + 4] + c[18 + 5];
    const double gd0 = c[3] + c[9 + 6] + c[18 + 7];
    const double gd1 = c[6] + c[9 + 4] + c[18 + 8];
    const double gd2 = c[7] + c[9 + 8] + c[18 + 5];
    vis[0] = 0.5 * lap0 + gd0 / 6.0;
    vis[1] = 0.5 * lap1 + gd1 / 6.0;
    vis[2] = 0.5 * lap2 + gd2 / 6.0;
}

// Handoff layout: [0,27) rows 0-2 of G^-1 (row-major 3x9), [27,33) gd,
// 33 div, [34,37) viscous terms.
__device__ __forceinline__ void store_hand(double* hand, int64_t n, int64_t i,
                                           const double (&ginv3)[27], bool has_ginv,
                                           const Closure& r, const double (&vis)[3])
{
    if (has_ginv) {
#pragma unroll
        for (int q = 0; q < 27; ++q) hand[(int64_t)q * n + i] = ginv3[q];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) hand[(int64_t)(27 + q) * n + i] = r.gd[q];
    hand[(int64_t)33 * n + i] = r.div;
#pragma unroll
    for (int q = 0; q < 3; ++q) hand[(int64_t)(34 + q) * n + i] = vis[q];
}

// rows 0-2 of G^{-1} from the factor, stored straight into the handoff
// (one row live at a time)
template <int N>
__device__ __forceinline__ void store_ginv_rows(const double (&U)[45], double* hand,
                                                int64_t n, int64_t i)
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double e[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) e[q] = (q == r) ? 1.0 : 0.0;
        chol_solve<N>(U, e);
#pragma unroll
        for (int q = 0; q < 9; ++q) hand[(int64_t)(r * 9 + q) * n + i] = (q < N) ? e[q] : 0.0;
    }
}

// rows 0-2 of G^{-1} from the factor (3 solves with unit vectors)
template <int N>
__device__ __forceinline__ void ginv_rows(const double (&U)[45], double out[27])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double e[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) e[q] = (q == r) ? 1.0 : 0.0;
        chol_solve<N>(U, e);
#pragma unroll
        for (int q = 0; q < 9; ++q) out[r * 9 + q] = (q < N) ? e[q] : 0.0;
    }
}

// Rows the fit's order decision sees: a stencil with fewer real (non-ghost)
// rows than min_real counts as having fewer than 9 rows, so it takes the
// linear fit, whatever its ghost rows add.
__device__ __forceinline__ int order_rows(const View& v, const Rec& r, int mt)
{
    return (r.m < v.min_real && mt >= 9) ? 8 : mt;
}

// Calls f(a, w, p) for every fit row of real particle i: the stencil rows
// (p = the stencil point) then the ghost rows in octant order (p = null).
// Returns the number of rows.
template <int B = FIT_BATCH, class F>
__device__ __forceinline__ int for_rows(const View& v, const GridInfo& g,
                                        int64_t i, const Rec& r, F&& f)
{
    int m = 0;
    visit_stencil<B>(v, g, i, r, [&](const Pt& p, double dx, double dy, double dz) {
        double a[9];
        const double w = point_row(v, g, dx, dy, dz, a);
        f(a, w, &p);
        ++m;
    });
#pragma unroll
    for (int o = 0; o < 8; ++o)
        if ((r.gm >> o) & 1) {
            double a[9];
            const double w = ghost_row(v, g, o, a);
            f(a, w, (const Pt*)nullptr);
            ++m;
        }
    return m;
}

// for_rows for a particle of a staged tile: stencil rows from the LDS
// copies (sx, sy, sz) through visit_staged, then the ghost rows.
// UNIT: the weights are unit (LP_W_UNIT), so f receives the constant 1.
template <int B, bool UNIT, class F>
__device__ __forceinline__ int for_rows_staged(const View& v, const GridInfo& g,
                                               int64_t i, const Rec& r, const double* sx,
                                               const double* sy, const double* sz, F&& f)
{
    int m = 0;
    const Seen s = seen_from(v, g, i);
    visit_staged<B>(v, s, i, r, sx, sy, sz,
                    [&](const Pt& p, double dx, double dy, double dz) {
        double a[9];
        const double w = point_row(v, g, dx, dy, dz, a);
        f(a, UNIT ? 1.0 : w, &p);
        ++m;
    });
#pragma unroll
    for (int o = 0; o < 8; ++o)
        if ((r.gm >> o) & 1) {
            double a[9];
            const double w = ghost_row(v, g, o, a);
            f(a, UNIT ? 1.0 : w, (const Pt*)nullptr);
            ++m;
        }
    return m;
}

// for_rows_staged with the rows spread over LPP adjacent lanes: lane sub
// takes the kept rows sub, sub + LPP, ... (visit_staged_sub) and the ghost
// rows o with o mod LPP = sub; returns this lane's rows.
template <int B, int LPP, bool UNIT, class F>
__device__ __forceinline__ int for_rows_staged_sub(const View& v, const GridInfo& g,
                                                   int64_t i, const Rec& r, int sub,
                                                   const double* sx, const double* sy,
                                                   const double* sz, F&& f)
{
    int m = 0;
    const Seen s = seen_from(v, g, i);
    visit_staged_sub<B, LPP>(v, s, i, r, sub, sx, sy, sz,
                             [&](const Pt& p, double dx, double dy, double dz) {
        double a[9];
        const double w = point_row(v, g, dx, dy, dz, a);
        f(a, UNIT ? 1.0 : w, &p);
        ++m;
    });
#pragma unroll
    for (int o = 0; o < 8; ++o)
        if (((r.gm >> o) & 1) && (o % LPP) == sub) {
            double a[9];
            const double w = ghost_row(v, g, o, a);
            f(a, UNIT ? 1.0 : w, (const Pt*)nullptr);
            ++m;
        }
    return m;
}

// for_rows with the rows spread over LPP lanes (stencil rows as in
// visit_stencil_sub, ghost o to lane o mod LPP; B: rows loaded together
// with one lane per particle); returns this lane's rows.
template <int LPP, int B = FIT_BATCH, class F>
__device__ __forceinline__ int for_rows_sub(const View& v, const GridInfo& g, int64_t i,
                                            const Rec& r, int sub, F&& f)
{
    if (LPP == 1) return for_rows<B>(v, g, i, r, f);
    int m = 0;
    visit_stencil_sub<LPP>(v, g, i, r, sub, [&](const Pt& p, double dx, double dy,
                                                double dz) {
        double a[9];
        const double w = point_row(v, g, dx, dy, dz, a);
        f(a, w, &p);
        ++m;
    });
#pragma unroll
    for (int o = 0; o < 8; ++o)
        if (((r.gm >> o) & 1) && (o % LPP) == sub) {
            double a[9];
            const double w = ghost_row(v, g, o, a);
            f(a, w, (const Pt*)nullptr);
            ++m;
        }
    return m;
}

// The Gram matrix of the Taylor rows a = (x, y, z, x^2/2, y^2/2, z^2/2,
// xy, xz, yz) has 31 distinct entries: the weighted sums of the monomials
// of degree 2, 3 and 4 in (x, y, z).  They are accumulated row by row
// (fewer registers and operations than the 45 products) and G is
// assembled once per particle.
//   0 xx 1 yy 2 zz 3 xy 4 xz 5 yz
//   6 xxx 7 yyy 8 zzz 9 xxy 10 xxz 11 xyy 12 yyz 13 xzz 14 yzz 15 xyz
//   16 xxxx 17 yyyy 18 zzzz 19 xxyy 20 xxzz 21 yyzz 22 xxxy 23 xxxz
//   24 xyyy 25 yyyz 26 xzzz 27 yzzz 28 xxyz 29 xyyz 30 xyzz
template <class T>
__device__ __forceinline__ void moments_add(T (&M)[31], const T* a, T w)
{
    const T x = a[0], y = a[1], z = a[2];
    const T xx = x * x, yy = y * y, zz = z * z;
    const T xy = a[6], xz = a[7], yz = a[8];
    const T wxx = w * xx, wyy = w * yy, wzz = w * zz, wxy = w * xy;
    M[0] += wxx;
    M[1] += wyy;
    M[2] += wzz;
    M[3] += wxy;
    M[4] += w * xz;
    M[5] += w * yz;
    M[6] += wxx * x;
    M[7] += wyy * y;
    M[8] += wzz * z;
    M[9] += wxx * y;
    M[10] += wxx * z;
    M[11] += wyy * x;
    M[12] += wyy * z;
    M[13] += wzz * x;
    M[14] += wzz * y;
    M[15] += wxy * z;
    M[16] += wxx * xx;
    M[17] += wyy * yy;
    M[18] += wzz * zz;
    M[19] += wxx * yy;
    M[20] += wxx * zz;
    M[21] += wyy * zz;
    M[22] += wxx * xy;
    M[23] += wxx * xz;
    M[24] += wyy * xy;
    M[25] += wyy * yz;
    M[26] += wzz * xz;
    M[27] += wzz * yz;
    M[28] += wxx * yz;
    M[29] += wyy * xz;
    M[30] += wzz * xy;
}

template <class T>
__device__ __forceinline__ void gram_from_moments(const T (&M)[31], T (&G)[45])
{
    // row 0: x
    G[uix(0, 0)] = M[0];  G[uix(0, 1)] = M[3];  G[uix(0, 2)] = M[4];
    G[uix(0, 3)] = T(0.5) * M[6];  G[uix(0, 4)] = T(0.5) * M[11];
    G[uix(0, 5)] = T(0.5) * M[13]; G[uix(0, 6)] = M[9];  G[uix(0, 7)] = M[10];
    G[uix(0, 8)] = M[15];
    // row 1: y
    G[uix(1, 1)] = M[1];  G[uix(1, 2)] = M[5];  G[uix(1, 3)] = T(0.5) * M[9];
    G[uix(1, 4)] = T(0.5) * M[7];  G[uix(1, 5)] = T(0.5) * M[14];
    G[uix(1, 6)] = M[11]; G[uix(1, 7)] = M[15]; G[uix(1, 8)] = M[12];
    // row 2: z
    G[uix(2, 2)] = M[2];  G[uix(2, 3)] = T(0.5) * M[10]; G[uix(2, 4)] = T(0.5) * M[12];
    G[uix(2, 5)] = T(0.5) * M[8];  G[uix(2, 6)] = M[15]; G[uix(2, 7)] = M[13];
    G[uix(2, 8)] = M[14];
    // row 3: x^2/2
    G[uix(3, 3)] = T(0.25) * M[16]; G[uix(3, 4)] = T(0.25) * M[19];
    G[uix(3, 5)] = T(0.25) * M[20]; G[uix(3, 6)] = T(0.5) * M[22];
    G[uix(3, 7)] = T(0.5) * M[23];  G[uix(3, 8)] = T(0.5) * M[28];
    // row 4: y^2/2
    G[uix(4, 4)] = T(0.25) * M[17]; G[uix(4, 5)] = T(0.25) * M[21];
    G[uix(4, 6)] = T(0.5) * M[24];  G[uix(4, 7)] = T(0.5) * M[29];
    G[uix(4, 8)] = T(0.5) * M[25];
    // row 5: z^2/2
    G[uix(5, 5)] = T(0.25) * M[18]; G[uix(5, 6)] = T(0.5) * M[30];
    G[uix(5, 7)] = T(0.5) * M[26];  G[uix(5, 8)] = T(0.5) * M[27];
    // rows 6-8: xy, xz, yz
    G[uix(6, 6)] = M[19]; G[uix(6, 7)] = M[28]; G[uix(6, 8)] = M[29];
    G[uix(7, 7)] = M[20]; G[uix(7, 8)] = M[30];
    G[uix(8, 8)] = M[21];
}

// P and eta carried by a row: reals their own, mirrors the pressure of
// their source's density at zero shear rate and no viscosity, ghosts 0.
__device__ __forceinline__ void pass2_values(const View& v, const double* P,
                                             const double* eta, const Pt* p,
                                             const lp_params& prm, double& Pj,
                                             double& Ej)
{
    if (!p) {
        Pj = 0.0;
        Ej = 0.0;
    } else if (!p->mirror) {
        Pj = P[p->src];
        Ej = eta[p->src];
    } else {
        const double Vs = v.V[p->src];
        Pj = mirror_pressure(prm, Vs);
        // hydrostatic wall pressure (option): plus the weight of the layer
        // between the mirror and its source
        if (v.wall_pressure)
            Pj = Pj + prm.rho_s * (1.0 / Vs) * (-prm.g[2]) * (v.z[p->src] - p->z);
        Ej = 0.0;
    }
}

// ---- staging of a tile's list sources in LDS (fits and their adjoints) --

// Staged sources per thread of a block of NT threads, and this thread's
// source ids in the tile (slot threadIdx.x + u NT; -1 past the tile's S
// sources).
template <int NT = BLOCK>
constexpr int stage_per() { return (STAGE_CAP + NT - 1) / NT; }
// six staged FP64 fields per source; two blocks must fit one CU's 160 KB
static_assert(2 * 6 * STAGE_CAP * (int)sizeof(double) <= 160 * 1024,
              "two staged fit blocks per CU");

template <int NT = BLOCK>
__device__ __forceinline__ void stage_ids(const View& v, int64_t tile, int S,
                                          int32_t (&js)[stage_per<NT>()])
{
    const int32_t* src = v.tile_src + tile * STAGE_CAP;
#pragma unroll
    for (int u = 0; u < stage_per<NT>(); ++u) {
        const int q = (int)threadIdx.x + u * NT;
        js[u] = q < S ? src[q] : -1;
    }
}

// Loads the positions and velocities of the tile's S list sources into
// LDS (slot q holds the q-th source of the tile's sorted set): every
// thread takes its sources at once, their ids first, then their fields.
template <int NT = BLOCK>
__device__ __forceinline__ void stage_pass1(const View& v, int64_t tile, int S, double* sx,
                                            double* sy, double* sz, double* su,
                                            double* sv, double* sw)
{
    constexpr int SP = stage_per<NT>();
    int32_t js[SP];
    stage_ids<NT>(v, tile, S, js);
    double f[6][SP];
#pragma unroll
    for (int u = 0; u < SP; ++u) {
        const int32_t j = js[u] < 0 ? 0 : js[u];
        f[0][u] = v.x[j];
        f[1][u] = v.y[j];
        f[2][u] = v.z[j];
        f[3][u] = v.u[j];
        f[4][u] = v.v[j];
        f[5][u] = v.w[j];
    }
#pragma unroll
    for (int u = 0; u < SP; ++u) {
        if (js[u] < 0) continue;
        const int q = (int)threadIdx.x + u * NT;
        sx[q] = f[0][u];
        sy[q] = f[1][u];
        sz[q] = f[2][u];
        su[q] = f[3][u];
        sv[q] = f[4][u];
        sw[q] = f[5][u];
    }
}

// Loads the positions, P and eta of the tile's S list sources into LDS,
// with the pressure a mirror of each source carries (pass2_values).
template <int NT = BLOCK>
__device__ __forceinline__ void stage_pass2(const View& v, const double* P,
                                            const double* eta, int64_t tile, int S,
                                            double* sx, double* sy, double* sz,
                                            double* sP, double* sE, double* sM)
{
    constexpr int SP = stage_per<NT>();
    int32_t js[SP];
    stage_ids<NT>(v, tile, S, js);
    double f[5][SP];
#pragma unroll
    for (int u = 0; u < SP; ++u) {
        const int32_t j = js[u] < 0 ? 0 : js[u];
        f[0][u] = v.x[j];
        f[1][u] = v.y[j];
        f[2][u] = v.z[j];
        f[3][u] = P[j];
        f[4][u] = eta[j];
    }
#pragma unroll
    for (int u = 0; u < SP; ++u) {
        if (js[u] < 0) continue;
        const int q = (int)threadIdx.x + u * NT;
        const int32_t j = js[u];
        sx[q] = f[0][u];
        sy[q] = f[1][u];
        sz[q] = f[2][u];
        sP[q] = f[3][u];
        sE[q] = f[4][u];
        // j's system is that of every particle listing it.  Only a source
        // within R of the wall has a mirror (the rule that sets mirror_of).
        const int sj = sys_of(v.off, v.n_sys, j);
        const GridInfo& gj = v.grid[sj];
        double pm = 0.0;
        if (dsub(f[2][u], gj.wall) < gj.R) {
            Pt m;
            m.mirror = true;
            m.src = j;
            m.z = dsub(dmul(2.0, gj.wall), f[2][u]);
            double em;
            pass2_values(v, P, eta, &m, v.prm[sj], pm, em);
        }
        sM[q] = pm;
    }
}

}  // namespace lp
