// Adjoint (reverse-mode derivative) of one LP step with its stencils,
// ghost masks, fallback choices and regime branches held fixed.
//
// The step differentiated re-sorts its input by the context's cells and
// then steps (lp_build_cells followed by lp_step): mirrors (Sec. 3.1 step 9),
// least squares for u, v, w (Sec. 3.1 step 7), mu(I) closure (Sec. 2.2,
// 2.2.1), least squares for P and eta, Form E right-hand side (Sec. 2.1),
// explicit update (Sec. 3.1 steps 8, 10).  Its reverse, in reverse order:
//
//   update:   xbar += x'bar, ubar += u'bar + dt x'bar, Vbar += V'bar,
//             abar = dt (u'bar + dt x'bar / 2), dVbar = dt V'bar
//             (the seeds of the reverse right-hand side; the two stages of
//             the second-order step use other linear seeds, see AdjSeed);
//   RHS:      a = V T / rho_s + g with T = -grad P + gd grad eta + eta vis,
//             dV/dt = V div;
//   a least-squares fit c = G^-1 A^T b (G = A^T A) with cbar:
//             y = G^-1 cbar, bbar_k = a_k . y,
//             Abar_k = r_k y - bbar_k c   (r = b - A c),
//             the rows a_k(xi) with xi = (x_k - x_i)/h carry Abar_k to the
//             positions of the row's point and of the particle;
//   closure:  derivatives of P = rho_s (k |gd|)^2 and
//             eta = rho_s mu(I) k^2 |gd| (inertial branch, k = 2 a d/(phi_c
//             - phi), I = (phi_c - phi)/a), P = rho_s (alpha + beta phi)
//             (quasi-static); dmu/dmu_s = I0/(I0 + I), dmu/dmu_2 =
//             I/(I0 + I), dmu/dI0 = -(mu_2 - mu_s) I/(I0 + I)^2.  The
//             shear-rate norm has zero derivative where it is zero.
//
// Contributions to other particles (neighbour values and positions,
// mirror sources) are written, one record of six doubles per stencil row,
// into slots grouped by receiving particle (a counting sort of the rows by
// their point, built once per call with integer atomics); a gather pass
// then adds each particle's slots.  The order of the slots of one particle
// varies between runs, so sums are accumulated in a run-dependent order.
#include <cmath>

#include "lp_fitcore.h"

namespace lp {

namespace {

inline unsigned int blocks_for(int64_t n, int per = BLOCK)
{
    return (unsigned int)((n + per - 1) / per);
}

struct Ptr7 {
    const double* p[7];
};

struct AdjBufs {
    double* a[7];        // accumulators: xbar ybar zbar ubar vbar wbar Vbar
    double* aP;          // Pbar
    double* aE;          // etabar
    double* stash;       // 11 x n: gdbar (6), divbar, visbar (3), own etabar
    const double* coefu; // 27 x n scaled velocity coefficients (forward)
    const double* P;
    const double* eta;
    const double* hand;  // forward handoff: gd (27..32), div (33), vis (34..36)
    const uint8_t* flags;
    double* dparams;     // n_sys x 3
    ErrWord* err;
    const int32_t* slot; // m_max x n: slot of stencil row t of particle i
    double* contrib;     // 6 per slot
};

// six contributions of one stencil row to the particle its point stands
// for (a mirror's source)
__device__ __forceinline__ void put_row(const AdjBufs& B, int64_t n, int64_t i, int t,
                                        double c0, double c1, double c2, double c3,
                                        double c4, double c5)
{
    const int64_t sl = B.slot[(int64_t)t * n + i];
    double2* q = reinterpret_cast<double2*>(B.contrib + 6 * sl);
    q[0] = make_double2(c0, c1);
    q[1] = make_double2(c2, c3);
    q[2] = make_double2(c4, c5);
}

// d(Taylor row)/d(xi) applied to a row cotangent Abar: returns xibar
__device__ __forceinline__ void row_xi_bar(const double (&A)[9], double ex, double ey,
                                           double ez, double& gx, double& gy,
                                           double& gz)
{
    gx = A[0] + A[3] * ex + A[6] * ey + A[7] * ez;
    gy = A[1] + A[4] * ey + A[6] * ex + A[8] * ez;
    gz = A[2] + A[5] * ez + A[7] * ex + A[8] * ey;
}

// zero records in the slots of particle i (a particle whose reverse step
// failed still owns its slots)
__device__ __forceinline__ void zero_rows(const AdjBufs& B, const View& v,
                                          const GridInfo& g, int64_t i, const Rec& r)
{
    int t = 0;
    visit_stencil(v, g, i, r, [&](const Pt&, double, double, double) {
        put_row(B, v.n, i, t, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0);
        ++t;
    });
}

// ---- slots: rows grouped by the particle they contribute to ------------

// cnt[j] = number of stencil rows (of all particles) whose point is j or
// a mirror of j
__global__ __launch_bounds__(BLOCK) void k_slot_count(View v, int32_t* cnt)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (i >= v.n) return;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    const Rec r = load_rec(v, i);
    visit_stencil(v, g, i, r, [&](const Pt& p, double, double, double) {
        atomicAdd(&cnt[p.src], 1);
    });
}

// exclusive scan of a[0..n) into b[0..n], tiles of BLOCK (three kernels)
__global__ __launch_bounds__(BLOCK) void k_scan_tiles(int64_t n, const int32_t* a,
                                                      int32_t* b, int32_t* tile)
{
    __shared__ int32_t ws[BLOCK / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t i = (int64_t)blockIdx.x * BLOCK + t;
    const int32_t x = i < n ? a[i] : 0;
    int32_t inc = x;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    int32_t pre = 0, tot = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
        if (w < wave) pre += ws[w];
        tot += ws[w];
    }
    if (i < n) b[i] = pre + inc - x;
    if (t == 0) tile[blockIdx.x] = tot;
}

__global__ void k_scan_tile_sums(int64_t nt, int32_t* tile)
{
    // single block of 1024: each thread scans a contiguous chunk
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (nt + 1023) / 1024;
    const int64_t b = t * chunk;
    const int64_t e = (b + chunk < nt) ? b + chunk : nt;
    int32_t sum = 0;
    for (int64_t q = b; q < e; ++q) sum += tile[q];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int32_t o = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += o;
        __syncthreads();
    }
    int32_t run = part[t] - sum;
    for (int64_t q = b; q < e; ++q) {
        const int32_t x = tile[q];
        tile[q] = run;
        run += x;
    }
    if (t == 1023) tile[nt] = part[1023];
}

__global__ void k_scan_add(int64_t n, int32_t* b, const int32_t* tile)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n) b[i] += tile[blockIdx.x];
    if (i == 0) b[n] = tile[(n + BLOCK - 1) / BLOCK];
}

// slot of every stencil row: start of its point's range plus a place
// taken with an atomic counter
__global__ __launch_bounds__(BLOCK) void k_slot_assign(View v, const int32_t* off,
                                                       int32_t* fill, int32_t* slot)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (i >= v.n) return;
    const int64_t n = v.n;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    const Rec r = load_rec(v, i);
    int t = 0;
    visit_stencil(v, g, i, r, [&](const Pt& p, double, double, double) {
        slot[(int64_t)t * n + i] = off[p.src] + atomicAdd(&fill[p.src], 1);
        ++t;
    });
}

__global__ void k_zero_i32(int64_t n, int32_t* a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

// adds the records of each particle's slots: pass 2 (P, eta, V, x, y, z)
// or pass 1 (u, v, w, x, y, z)
__global__ __launch_bounds__(BLOCK) void k_slot_gather(int64_t n, const int32_t* off,
                                                       AdjBufs B, int pass)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double c[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int32_t e = off[j + 1];
    for (int32_t sl = off[j]; sl < e; ++sl) {
        const double2* q = reinterpret_cast<const double2*>(B.contrib + 6 * (int64_t)sl);
        const double2 a = q[0], b = q[1], d = q[2];
        c[0] += a.x;
        c[1] += a.y;
        c[2] += b.x;
        c[3] += b.y;
        c[4] += d.x;
        c[5] += d.y;
    }
    if (pass == 2) {
        B.aP[j] += c[0];
        B.aE[j] += c[1];
        B.a[6][j] += c[2];
    } else {
        B.a[3][j] += c[0];
        B.a[4][j] += c[1];
        B.a[5][j] += c[2];
    }
    B.a[0][j] += c[3];
    B.a[1][j] += c[4];
    B.a[2][j] += c[5];
}

// N = nA A + nB B at particle i, component a (B optional)
__device__ __forceinline__ double seed_n(const AdjSeed& S, int a, int64_t i)
{
    const double v = S.nA * S.A[a][i];
    return S.B[0] ? v + S.nB * S.B[a][i] : v;
}

__global__ void k_adj_init(int64_t n, AdjSeed S, AdjBufs B)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double id[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
        const double v = S.iA * S.A[a][i];
        id[a] = S.B[0] ? v + S.iB * S.B[a][i] : v;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        B.a[a][i] = id[a];
        B.a[3 + a][i] = id[3 + a] + S.c_ux * seed_n(S, a, i);
    }
    B.a[6][i] = id[6];
    B.aP[i] = 0.0;
    B.aE[i] = 0.0;
}

// ---- reverse of the update, the RHS and the fit of P and eta -------------

__global__ __launch_bounds__(BLOCK) void k_adj_pass2(View v, AdjSeed S, AdjBufs B)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (i >= v.n) return;
    const int64_t n = v.n;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const lp_params& prm = v.prm[s];
    const Rec r = load_rec(v, i);
    const bool lin = B.flags[i] & FLAG_LINEAR;
    const double Pi = B.P[i], Ei = B.eta[i];
    // forward fit of P and eta (all nine coefficients)
    double M[31], y0[9], y1[9];
#pragma unroll
    for (int q = 0; q < 31; ++q) M[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) y0[q] = y1[q] = 0.0;
    for_rows(v, g, i, r, [&](const double* a, double w, const Pt* p) {
        moments_add(M, a, w);
        double Pj, Ej;
        pass2_values(v, B.P, B.eta, p, prm, Pj, Ej);
        const double bP = w * (Pj - Pi), bE = w * (Ej - Ei);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            y0[q] += a[q] * bP;
            y1[q] += a[q] * bE;
        }
    });
    double U[45];
    gram_from_moments(M, U);
    const double ratio = lin ? cholesky<3>(U) : cholesky<9>(U);
    if (!(ratio > 0.0)) {
        raise_error(B.err, ERR_NUMERIC, i);
        for (int q = 0; q < 11; ++q) B.stash[(int64_t)q * n + i] = 0.0;
        zero_rows(B, v, g, i, r);
        return;
    }
    double cP[9], cE[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        cP[q] = (lin && q >= 3) ? 0.0 : y0[q];
        cE[q] = (lin && q >= 3) ? 0.0 : y1[q];
    }
    if (lin) {
        chol_solve<3>(U, cP);
        chol_solve<3>(U, cE);
    } else {
        chol_solve<9>(U, cP);
        chol_solve<9>(U, cE);
    }
    const double ih = g.inv_h;
    double gP[3], gE[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        gP[a] = cP[a] * ih;
        gE[a] = cE[a] * ih;
    }
    // handoff of the forward closure
    double gd[6], vis[3];
#pragma unroll
    for (int q = 0; q < 6; ++q) gd[q] = B.hand[(int64_t)(27 + q) * n + i];
    const double div = B.hand[(int64_t)33 * n + i];
#pragma unroll
    for (int q = 0; q < 3; ++q) vis[q] = B.hand[(int64_t)(34 + q) * n + i];
    // ---- reverse of the update and the RHS (this particle's own terms)
    const double V = v.V[i];
    double abar[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
        abar[a] = S.c_a * (seed_n(S, 3 + a, i) + S.k_x * seed_n(S, a, i));
    const double dVbar = S.c_d * seed_n(S, 6, i);
    const double T0 = -gP[0] + gd[0] * gE[0] + gd[3] * gE[1] + gd[4] * gE[2] + Ei * vis[0];
    const double T1 = -gP[1] + gd[3] * gE[0] + gd[1] * gE[1] + gd[5] * gE[2] + Ei * vis[1];
    const double T2 = -gP[2] + gd[4] * gE[0] + gd[5] * gE[1] + gd[2] * gE[2] + Ei * vis[2];
    const double inv_rho = 1.0 / prm.rho_s;
    B.a[6][i] += (abar[0] * T0 + abar[1] * T1 + abar[2] * T2) * inv_rho + dVbar * div;
    const double Tb[3] = {abar[0] * V * inv_rho, abar[1] * V * inv_rho,
                          abar[2] * V * inv_rho};
    double gPb[3], gEb[3];
    gPb[0] = -Tb[0];
    gPb[1] = -Tb[1];
    gPb[2] = -Tb[2];
    gEb[0] = Tb[0] * gd[0] + Tb[1] * gd[3] + Tb[2] * gd[4];
    gEb[1] = Tb[0] * gd[3] + Tb[1] * gd[1] + Tb[2] * gd[5];
    gEb[2] = Tb[0] * gd[4] + Tb[1] * gd[5] + Tb[2] * gd[2];
    double* st = B.stash;
    st[(int64_t)0 * n + i] = Tb[0] * gE[0];
    st[(int64_t)1 * n + i] = Tb[1] * gE[1];
    st[(int64_t)2 * n + i] = Tb[2] * gE[2];
    st[(int64_t)3 * n + i] = Tb[0] * gE[1] + Tb[1] * gE[0];
    st[(int64_t)4 * n + i] = Tb[0] * gE[2] + Tb[2] * gE[0];
    st[(int64_t)5 * n + i] = Tb[1] * gE[2] + Tb[2] * gE[1];
    st[(int64_t)6 * n + i] = dVbar * V;
#pragma unroll
    for (int a = 0; a < 3; ++a) st[(int64_t)(7 + a) * n + i] = Ei * Tb[a];
    st[(int64_t)10 * n + i] = Tb[0] * vis[0] + Tb[1] * vis[1] + Tb[2] * vis[2];
    // ---- reverse of the fit of P and eta
    double yP[9], yE[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        yP[q] = q < 3 ? gPb[q] * ih : 0.0;
        yE[q] = q < 3 ? gEb[q] * ih : 0.0;
    }
    if (lin) {
        chol_solve<3>(U, yP);
        chol_solve<3>(U, yE);
    } else {
        chol_solve<9>(U, yP);
        chol_solve<9>(U, yE);
    }
    double sP = 0.0, sE = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    int t = 0;
    for_rows(v, g, i, r, [&](const double* a, double w, const Pt* p) {
        double Pj, Ej;
        pass2_values(v, B.P, B.eta, p, prm, Pj, Ej);
        double rP = Pj - Pi, rE = Ej - Ei, bP = 0.0, bE = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            rP -= a[q] * cP[q];
            rE -= a[q] * cE[q];
            bP += a[q] * yP[q];
            bE += a[q] * yE[q];
        }
        sP -= bP;
        sE -= bE;
        if (!p) return;   // ghost rows: constant rows, value 0
        double Ab[9];
#pragma unroll
        for (int q = 0; q < 9; ++q)
            Ab[q] = rP * yP[q] - bP * cP[q] + rE * yE[q] - bE * cE[q];
        double gx, gy, gz;
        row_xi_bar(Ab, a[0], a[1], a[2], gx, gy, gz);
        gx *= ih;
        gy *= ih;
        gz *= ih;
        sx -= gx;
        sy -= gy;
        sz -= gz;
        if (!p->mirror) {
            put_row(B, n, i, t, bP, bE, 0.0, gx, gy, gz);
        } else {
            // mirror pressure P(phi_src) of the quasi-static law; no eta
            const double Vs = v.V[p->src];
            const double dV = 1.0 / Vs > prm.phi_max
                                  ? -bP * prm.rho_s * prm.beta / (Vs * Vs) : 0.0;
            put_row(B, n, i, t, 0.0, 0.0, dV, gx, gy, -gz);
        }
        ++t;
    });
    // this particle's own terms: no other thread writes them in this pass
    B.aP[i] += sP;
    B.aE[i] += sE;
    B.a[0][i] += sx;
    B.a[1][i] += sy;
    B.a[2][i] += sz;
}

// ---- reverse of the closure and of the fit of u, v, w ----------------------

__global__ __launch_bounds__(BLOCK) void k_adj_pass1(View v, AdjBufs B)
{
    __shared__ double red[3][BLOCK];
    const int t = threadIdx.x;
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + t;
    double th[3] = {0.0, 0.0, 0.0};
    int s = -1;
    if (i < v.n) {
        const int64_t n = v.n;
        s = sys_of(v.off, v.n_sys, i);
        const GridInfo& g = v.grid[s];
        const lp_params& prm = v.prm[s];
        const Rec r = load_rec(v, i);
        const bool lin = B.flags[i] & FLAG_LINEAR;
        double c[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) c[q] = B.coefu[(int64_t)q * n + i];
        const double V = v.V[i];
        const Closure cl = closure(prm, V, c);
        // cotangents arriving at this particle's closure outputs
        const double* st = B.stash;
        double gdb[6], visb[3];
#pragma unroll
        for (int q = 0; q < 6; ++q) gdb[q] = st[(int64_t)q * n + i];
        double divb = st[(int64_t)6 * n + i];
#pragma unroll
        for (int q = 0; q < 3; ++q) visb[q] = st[(int64_t)(7 + q) * n + i];
        const double Pb = B.aP[i];
        const double Eb = B.aE[i] + st[(int64_t)10 * n + i];
        // ---- closure
        double phib = 0.0, gnb = 0.0;
        const double phi = 1.0 / V;
        if (cl.branch == 1) {
            const double a = prm.phi_c - prm.phi_min;
            const double wd = prm.phi_c - phi;
            const double k = 2.0 * a * prm.d / wd;
            const double gn = cl.gn, I = cl.I, mu = cl.mu;
            gnb = Pb * 2.0 * prm.rho_s * k * k * gn + Eb * prm.rho_s * mu * k * k;
            const double mub = Eb * prm.rho_s * k * k * gn;
            const double kb = Pb * 2.0 * prm.rho_s * k * gn * gn +
                              Eb * 2.0 * prm.rho_s * mu * k * gn;
            const double den = prm.I0 + I;
            const double Ib = mub * (prm.mu_2 - prm.mu_s) * prm.I0 / (den * den);
            phib = kb * 2.0 * a * prm.d / (wd * wd) - Ib / a;
            th[0] = mub * prm.I0 / den;
            th[1] = mub * I / den;
            th[2] = -mub * (prm.mu_2 - prm.mu_s) * I / (den * den);
        } else if (cl.branch == 2) {
            phib = Pb * prm.rho_s * prm.beta;
        }
        B.a[6][i] += -phib / (V * V);
        if (cl.gn > 0.0) {
            const double q = gnb / cl.gn;
            gdb[0] += 0.5 * q * cl.gd[0];
            gdb[1] += 0.5 * q * cl.gd[1];
            gdb[2] += 0.5 * q * cl.gd[2];
            gdb[3] += q * cl.gd[3];
            gdb[4] += q * cl.gd[4];
            gdb[5] += q * cl.gd[5];
        }
        // gd and div from the velocity gradient, vis from its second
        // derivatives (coefficient index f*9 + q)
        double cb[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) cb[q] = 0.0;
        divb -= (gdb[0] + gdb[1] + gdb[2]) / 3.0;
        cb[0] += gdb[0] + divb;
        cb[10] += gdb[1] + divb;
        cb[20] += gdb[2] + divb;
        cb[1] += 0.5 * gdb[3];
        cb[9] += 0.5 * gdb[3];
        cb[2] += 0.5 * gdb[4];
        cb[18] += 0.5 * gdb[4];
        cb[11] += 0.5 * gdb[5];
        cb[19] += 0.5 * gdb[5];
        const double sixth = 1.0 / 6.0;
        cb[3] += 0.5 * visb[0] + sixth * visb[0];
        cb[4] += 0.5 * visb[0];
        cb[5] += 0.5 * visb[0];
        cb[15] += sixth * visb[0];
        cb[25] += sixth * visb[0];
        cb[12] += 0.5 * visb[1];
        cb[13] += 0.5 * visb[1] + sixth * visb[1];
        cb[14] += 0.5 * visb[1];
        cb[6] += sixth * visb[1];
        cb[26] += sixth * visb[1];
        cb[21] += 0.5 * visb[2];
        cb[22] += 0.5 * visb[2];
        cb[23] += 0.5 * visb[2] + sixth * visb[2];
        cb[7] += sixth * visb[2];
        cb[17] += sixth * visb[2];
        // ---- reverse of the fit of u, v, w (coefficients per unit h)
        const double ih = g.inv_h, ih2 = g.inv_h * g.inv_h;
        const double hh = g.h, hh2 = g.h * g.h;
        double M[31];
#pragma unroll
        for (int q = 0; q < 31; ++q) M[q] = 0.0;
        for_rows(v, g, i, r, [&](const double* a, double w, const Pt*) {
            moments_add(M, a, w);
        });
        double U[45];
        gram_from_moments(M, U);
        const double ratio = lin ? cholesky<3>(U) : cholesky<9>(U);
        if (!(ratio > 0.0)) {
            raise_error(B.err, ERR_NUMERIC, i);
            zero_rows(B, v, g, i, r);
        } else {
            double y[3][9], cu[3][9];
#pragma unroll
            for (int f = 0; f < 3; ++f) {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const bool on = !(lin && q >= 3);
                    y[f][q] = on ? cb[f * 9 + q] * (q < 3 ? ih : ih2) : 0.0;
                    cu[f][q] = on ? c[f * 9 + q] * (q < 3 ? hh : hh2) : 0.0;
                }
                if (lin) chol_solve<3>(U, y[f]);
                else chol_solve<9>(U, y[f]);
            }
            const double ui = v.u[i], vi = v.v[i], wi = v.w[i];
            double su[3] = {0.0, 0.0, 0.0}, sx = 0.0, sy = 0.0, sz = 0.0;
            int t = 0;
            for_rows(v, g, i, r, [&](const double* a, double w, const Pt* p) {
                double b[3] = {0.0, 0.0, 0.0};   // ghosts carry u_i
                if (p) {
                    double uj, vj, wj;
                    point_velocity(v, *p, uj, vj, wj);
                    b[0] = uj - ui;
                    b[1] = vj - vi;
                    b[2] = wj - wi;
                }
                double Ab[9];
#pragma unroll
                for (int q = 0; q < 9; ++q) Ab[q] = 0.0;
                double bb[3];
#pragma unroll
                for (int f = 0; f < 3; ++f) {
                    double rr = b[f], yy = 0.0;
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        rr -= a[q] * cu[f][q];
                        yy += a[q] * y[f][q];
                    }
                    bb[f] = yy;
#pragma unroll
                    for (int q = 0; q < 9; ++q) Ab[q] += rr * y[f][q] - yy * cu[f][q];
                }
                if (!p) return;   // ghost rows: constant, value u_i
                su[0] -= bb[0];
                su[1] -= bb[1];
                su[2] -= bb[2];
                double gx, gy, gz;
                row_xi_bar(Ab, a[0], a[1], a[2], gx, gy, gz);
                gx *= ih;
                gy *= ih;
                gz *= ih;
                sx -= gx;
                sy -= gy;
                sz -= gz;
                const double sg = p->mirror ? -1.0 : 1.0;
                put_row(B, n, i, t, bb[0], bb[1], sg * bb[2], gx, gy, sg * gz);
                ++t;
            });
            B.a[3][i] += su[0];
            B.a[4][i] += su[1];
            B.a[5][i] += su[2];
            B.a[0][i] += sx;
            B.a[1][i] += sy;
            B.a[2][i] += sz;
        }
    }
    // parameter cotangents: one atomic per block when the block lies in
    // one system, else one per thread
    __shared__ int sys_t[BLOCK];
    sys_t[t] = s;
    __syncthreads();
    const int s0 = sys_t[0];
    const bool uniform = __syncthreads_and((s == s0 || s < 0) ? 1 : 0) != 0 && s0 >= 0;
    if (uniform) {
        red[0][t] = th[0];
        red[1][t] = th[1];
        red[2][t] = th[2];
        __syncthreads();
        for (int w = BLOCK / 2; w > 0; w >>= 1) {
            if (t < w) {
                red[0][t] += red[0][t + w];
                red[1][t] += red[1][t + w];
                red[2][t] += red[2][t + w];
            }
            __syncthreads();
        }
        if (t == 0)
            for (int q = 0; q < 3; ++q) atomicAdd(&B.dparams[3 * s0 + q], red[q][0]);
    } else if (s >= 0) {
        for (int q = 0; q < 3; ++q)
            if (th[q] != 0.0) atomicAdd(&B.dparams[3 * s + q], th[q]);
    }
}

// adj_in[perm[j]] = acc[j] (perm null: adj_in[j] = acc[j])
__global__ void k_adj_unpermute(int64_t n, const int32_t* perm, AdjBufs B, Ptr7 out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t o = perm ? perm[j] : j;
#pragma unroll
    for (int a = 0; a < 7; ++a) const_cast<double*>(out.p[a])[o] = B.a[a][j];
}

}  // namespace

lp_status step_adjoint(lp_ctx* c, const double* const st[7], const AdjSeed& seed,
                       double* const out[7], double* dparams, const int32_t* perm)
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (n == 0) return LP_OK;
    View v = make_view(c, st);
    AdjBufs B;
    for (int a = 0; a < 7; ++a) B.a[a] = w.adj[a];
    B.aP = w.adj_P;
    B.aE = w.adj_E;
    B.stash = w.adj_stash;
    B.coefu = w.coefu;
    B.P = w.P;
    B.eta = w.eta;
    B.hand = w.hand;
    B.flags = w.flags;
    B.dparams = dparams;
    B.err = w.err;
    Ptr7 dout;
    for (int a = 0; a < 7; ++a) dout.p[a] = out[a];
    // slots of the stencil rows, grouped by receiving particle
    hipStream_t s = c->stream;
    const int64_t nt = (n + BLOCK - 1) / BLOCK;
    B.slot = w.adj_slot;
    B.contrib = w.adj_contrib;
    hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, w.adj_cnt);
    hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, w.adj_fill);
    hipLaunchKernelGGL(k_slot_count, dim3(blocks_for(n)), dim3(BLOCK), 0, s, v, w.adj_cnt);
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(BLOCK), 0, s, n, w.adj_cnt,
                       w.adj_off, w.adj_tile);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(1024), 0, s, nt, w.adj_tile);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nt), dim3(BLOCK), 0, s, n, w.adj_off,
                       w.adj_tile);
    hipLaunchKernelGGL(k_slot_assign, dim3(blocks_for(n)), dim3(BLOCK), 0, s, v,
                       w.adj_off, w.adj_fill, w.adj_slot);
    hipLaunchKernelGGL(k_adj_init, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, seed, B);
    hipLaunchKernelGGL(k_adj_pass2, dim3(blocks_for(n)), dim3(BLOCK), 0, s, v, seed, B);
    hipLaunchKernelGGL(k_slot_gather, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n,
                       (const int32_t*)w.adj_off, B, 2);
    hipLaunchKernelGGL(k_adj_pass1, dim3(blocks_for(n)), dim3(BLOCK), 0, s, v, B);
    hipLaunchKernelGGL(k_slot_gather, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n,
                       (const int32_t*)w.adj_off, B, 1);
    hipLaunchKernelGGL(k_adj_unpermute, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, perm, B,
                       dout);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "adjoint launch");
    return LP_OK;
}

}  // namespace lp
