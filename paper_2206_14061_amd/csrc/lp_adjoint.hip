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
// mirror sources), six per stencil row, are summed per tile: a block of
// BLOCK particles whose neighbours are staged in LDS (the tile map's
// sources) adds each row into LDS accumulators of the row's source slot,
// then adds every slot once into the receiving particle's global
// accumulators with float64 atomics; rows that are not staged add into
// global memory directly.  Atomics make the summation order vary between
// runs (results agree to rounding).
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
    double* recv;        // 6 x n: contributions received from other particles
    double* M;           // 31 x n: Gram moments of each particle's stencil rows
                         // (written by the reverse pass 2, read by pass 1)
};

// LDS accumulators of a tile's staged sources: six per source slot
constexpr int NRECV = 6;

// Lanes per particle in the two reverse kernels: their LDS (staged
// sources and accumulators) fills a CU, so a block of BLOCK particles on
// two lanes each puts two waves on every SIMD instead of one.
#ifndef LP_ADJ_LPP
#define LP_ADJ_LPP 2
#endif
constexpr int ADJ_LPP = LP_ADJ_LPP;

__device__ __forceinline__ void lds_add(double* p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Six contributions of one stencil row to the particle its point stands
// for (a mirror's source): into the tile's accumulators of slot q when
// the row was read from the staged sources, else into global memory
// (receiver j).
__device__ __forceinline__ void deliver(const AdjBufs& B, int64_t n, double* acc,
                                        bool staged, int32_t q_or_j, const double (&c)[6])
{
    if (staged) {
#pragma unroll
        for (int f = 0; f < NRECV; ++f) lds_add(acc + f * STAGE_CAP + q_or_j, c[f]);
    } else {
#pragma unroll
        for (int f = 0; f < NRECV; ++f) unsafeAtomicAdd(B.recv + f * n + q_or_j, c[f]);
    }
}

// Zeroes the accumulators of the tile's ns staged slots (NT threads).
template <int NT>
__device__ __forceinline__ void acc_zero(double* acc, int ns)
{
    for (int q = threadIdx.x; q < ns; q += NT)
#pragma unroll
        for (int f = 0; f < NRECV; ++f) acc[f * STAGE_CAP + q] = 0.0;
}

// Adds every staged slot's accumulators into its particle's global
// accumulators (after the block's rows are done; NT threads).
template <int NT>
__device__ __forceinline__ void acc_flush(const AdjBufs& B, int64_t n, const double* acc,
                                          const int32_t* tsrc, int ns)
{
    for (int q = threadIdx.x; q < ns; q += NT) {
        const int64_t j = tsrc[q];
#pragma unroll
        for (int f = 0; f < NRECV; ++f) {
            const double x = acc[f * STAGE_CAP + q];
            if (x != 0.0) unsafeAtomicAdd(B.recv + f * n + j, x);
        }
    }
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

// adds the contributions received in pass 2 (P, eta, V, x, y, z) to the
// accumulators and clears the receive buffers for pass 1
__global__ __launch_bounds__(BLOCK) void k_fold2(int64_t n, AdjBufs B)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double* r = B.recv;
    double v[NRECV];
#pragma unroll
    for (int f = 0; f < NRECV; ++f) v[f] = r[f * n + j];
    B.aP[j] += v[0];
    B.aE[j] += v[1];
    B.a[6][j] += v[2];
    B.a[0][j] += v[3];
    B.a[1][j] += v[4];
    B.a[2][j] += v[5];
#pragma unroll
    for (int f = 0; f < NRECV; ++f) r[f * n + j] = 0.0;
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
    // the receive buffers start empty for the reverse pass 2
#pragma unroll
    for (int f = 0; f < NRECV; ++f) B.recv[f * n + i] = 0.0;
}

// ---- reverse of the update, the RHS and the fit of P and eta -------------

// The stencil rows of particle i with the P and eta their points carry:
// from the tile's sources staged in LDS (positions, P, eta and mirror
// pressure, as the forward pass-2 fit reads them) when the tile is
// staged, else from global memory.  body(a, w, p, Pj, Ej, src): src is the
// real particle behind the point (a mirror's source).
// With LPP lanes per particle, lane sub visits its share of the rows.
template <int LPP, class F>
__device__ __forceinline__ void adj_rows2(const View& v, const GridInfo& g,
                                          const lp_params& prm, const AdjBufs& B,
                                          int64_t i, const Rec& r, int sub, bool staged,
                                          const int32_t* tsrc, const double* sx,
                                          const double* sy, const double* sz,
                                          const double* sP, const double* sE,
                                          const double* sM, F&& body)
{
    if (staged) {
        for_rows_staged_sub<FIT_BATCH, LPP, true>(v, g, i, r, sub, sx, sy, sz,
                                                  [&](const double* a, double w,
                                                      const Pt* p) {
            if (!p) body(a, w, p, 0.0, 0.0, -1);
            else if (p->mirror) body(a, w, p, sM[p->src], 0.0, tsrc[p->src]);
            else body(a, w, p, sP[p->src], sE[p->src], tsrc[p->src]);
        });
    } else {
        for_rows_sub<LPP>(v, g, i, r, sub, [&](const double* a, double w, const Pt* p) {
            double Pj, Ej;
            pass2_values(v, B.P, B.eta, p, prm, Pj, Ej);
            body(a, w, p, Pj, Ej, p ? p->src : -1);
        });
    }
}

// Reverse of the update, the RHS and the fit of P and eta at real particle
// i of the block's tile (ns staged sources, -1: not staged), on LPP
// adjacent lanes: each sums its share of the rows (lane sub), the sums are
// added across the lanes, every lane then solves the same small systems,
// and lane 0 writes the particle's own results.
template <int LPP>
__device__ __forceinline__ void adj2_particle(const View& v, const AdjSeed& S,
                                              const AdjBufs& B, int64_t tile, int64_t i,
                                              int sub, int ns, const double* sx,
                                              const double* sy, const double* sz,
                                              const double* sP, const double* sE,
                                              const double* sM, double* acc)
{
    const int64_t n = v.n;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const lp_params& prm = v.prm[s];
    const Rec r = load_rec(v, i);
    const bool staged = ns >= 0 && !(r.mode & MODE_SORTED);
    const int32_t* tsrc = v.tile_src + tile * STAGE_CAP;
    const bool lin = B.flags[i] & FLAG_LINEAR;
    const double Pi = B.P[i], Ei = B.eta[i];
    // forward fit of P and eta (all nine coefficients)
    double M[31], y0[9], y1[9];
#pragma unroll
    for (int q = 0; q < 31; ++q) M[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) y0[q] = y1[q] = 0.0;
    adj_rows2<LPP>(v, g, prm, B, i, r, sub, staged, tsrc, sx, sy, sz, sP, sE, sM,
                   [&](const double* a, double w, const Pt*, double Pj, double Ej,
                       int32_t) {
        moments_add(M, a, w);
        const double bP = w * (Pj - Pi), bE = w * (Ej - Ei);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            y0[q] += a[q] * bP;
            y1[q] += a[q] * bE;
        }
    });
    if (LPP > 1) {
#pragma unroll
        for (int q = 0; q < 31; ++q) M[q] = lane_sum<LPP>(M[q]);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            y0[q] = lane_sum<LPP>(y0[q]);
            y1[q] = lane_sum<LPP>(y1[q]);
        }
    }
    const bool lead = sub == 0;
    // the moments are those of the u, v, w fit too (same rows, unit
    // weights): the reverse pass 1 reads them instead of summing its rows
    if (lead) {
#pragma unroll
        for (int q = 0; q < 31; ++q) B.M[(int64_t)q * n + i] = M[q];
    }
    double U[45];
    gram_from_moments(M, U);
    const double ratio = lin ? cholesky<3>(U) : cholesky<9>(U);
    if (!(ratio > 0.0)) {
        if (lead) {
            raise_error(B.err, ERR_NUMERIC, i);
            for (int q = 0; q < 11; ++q) B.stash[(int64_t)q * n + i] = 0.0;
        }
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
    if (lead) B.a[6][i] += (abar[0] * T0 + abar[1] * T1 + abar[2] * T2) * inv_rho + dVbar * div;
    const double Tb[3] = {abar[0] * V * inv_rho, abar[1] * V * inv_rho,
                          abar[2] * V * inv_rho};
    double gPb[3], gEb[3];
    gPb[0] = -Tb[0];
    gPb[1] = -Tb[1];
    gPb[2] = -Tb[2];
    gEb[0] = Tb[0] * gd[0] + Tb[1] * gd[3] + Tb[2] * gd[4];
    gEb[1] = Tb[0] * gd[3] + Tb[1] * gd[1] + Tb[2] * gd[5];
    gEb[2] = Tb[0] * gd[4] + Tb[1] * gd[5] + Tb[2] * gd[2];
    if (lead) {
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
    }
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
    double aPs = 0.0, aEs = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    adj_rows2<LPP>(v, g, prm, B, i, r, sub, staged, tsrc, sx, sy, sz, sP, sE, sM,
                   [&](const double* a, double, const Pt* p, double Pj, double Ej,
                       int32_t src) {
        double rP = Pj - Pi, rE = Ej - Ei, bP = 0.0, bE = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            rP -= a[q] * cP[q];
            rE -= a[q] * cE[q];
            bP += a[q] * yP[q];
            bE += a[q] * yE[q];
        }
        aPs -= bP;
        aEs -= bE;
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
        ax -= gx;
        ay -= gy;
        az -= gz;
        if (!p->mirror) {
            const double c[6] = {bP, bE, 0.0, gx, gy, gz};
            deliver(B, n, acc, staged, staged ? p->src : src, c);
        } else {
            // mirror pressure P(phi_src) of the quasi-static law; no eta
            const double Vs = v.V[src];
            const double dV = 1.0 / Vs > prm.phi_max
                                  ? -bP * prm.rho_s * prm.beta / (Vs * Vs) : 0.0;
            const double c[6] = {0.0, 0.0, dV, gx, gy, -gz};
            deliver(B, n, acc, staged, staged ? p->src : src, c);
        }
    });
    // this particle's own terms (other particles' rows arrive in B.recv)
    if (LPP > 1) {
        aPs = lane_sum<LPP>(aPs);
        aEs = lane_sum<LPP>(aEs);
        ax = lane_sum<LPP>(ax);
        ay = lane_sum<LPP>(ay);
        az = lane_sum<LPP>(az);
    }
    if (lead) {
        B.aP[i] += aPs;
        B.aE[i] += aEs;
        B.a[0][i] += ax;
        B.a[1][i] += ay;
        B.a[2][i] += az;
    }
}

// One block per tile: the tile's sources staged in LDS with their
// accumulators (all the LDS of a CU), the reverse pass of each particle
// (LPP lanes each), then the accumulators added into the global receive
// buffers.
template <int LPP>
__global__ __launch_bounds__(BLOCK * LPP, 1) void k_adj_pass2(View v, AdjSeed S, AdjBufs B,
                                                              int map_ok)
{
    constexpr int NT = BLOCK * LPP;
    __shared__ double sx[STAGE_CAP], sy[STAGE_CAP], sz[STAGE_CAP];
    __shared__ double sP[STAGE_CAP], sE[STAGE_CAP], sM[STAGE_CAP];
    __shared__ double acc[NRECV * STAGE_CAP];
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = tile * BLOCK + threadIdx.x / LPP;
    const int sub = threadIdx.x % LPP;
    const int tc = map_ok ? v.tile_cnt[tile] : -1;
    const int ns = tc <= STAGE_CAP ? tc : -1;   // -1: not staged
    if (ns >= 0) {
        stage_pass2<NT>(v, B.P, B.eta, tile, ns, sx, sy, sz, sP, sE, sM);
        acc_zero<NT>(acc, ns);
        __syncthreads();
    }
    if (i < v.n) adj2_particle<LPP>(v, S, B, tile, i, sub, ns, sx, sy, sz, sP, sE, sM, acc);
    if (ns >= 0) {
        __syncthreads();
        acc_flush<NT>(B, v.n, acc, v.tile_src + tile * STAGE_CAP, ns);
    }
}

// ---- reverse of the closure and of the fit of u, v, w ----------------------

// LPP lanes per particle, as in k_adj_pass2.
template <int LPP>
__global__ __launch_bounds__(BLOCK * LPP, 1) void k_adj_pass1(View v, AdjBufs B, int map_ok)
{
    constexpr int NT = BLOCK * LPP;
    // the tile's staged sources (positions and velocities, as the forward
    // pass-1 fit reads them) and their accumulators (all the LDS of a CU);
    // the block reduction of the parameter cotangents reuses the staging
    // space once every row has been read
    __shared__ double lds[6 * STAGE_CAP];
    __shared__ double acc[NRECV * STAGE_CAP];
    __shared__ int sys_t[NT];
    static_assert(3 * NT <= 6 * STAGE_CAP, "reduction fits the staging space");
    double* sx = lds;
    double* sy = lds + STAGE_CAP;
    double* sz = lds + 2 * STAGE_CAP;
    double* su = lds + 3 * STAGE_CAP;
    double* sv = lds + 4 * STAGE_CAP;
    double* sw = lds + 5 * STAGE_CAP;
    const int t = threadIdx.x;
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = tile * BLOCK + t / LPP;
    const int sub = t % LPP;
    const bool lead = sub == 0;
    const int tc = map_ok ? v.tile_cnt[tile] : -1;
    const int ns = tc <= STAGE_CAP ? tc : -1;   // -1: not staged
    if (ns >= 0) {
        stage_pass1<NT>(v, tile, ns, sx, sy, sz, su, sv, sw);
        acc_zero<NT>(acc, ns);
        __syncthreads();
    }
    double th[3] = {0.0, 0.0, 0.0};
    int s = -1;
    if (i < v.n) {
        const int64_t n = v.n;
        s = sys_of(v.off, v.n_sys, i);
        const GridInfo& g = v.grid[s];
        const lp_params& prm = v.prm[s];
        const Rec r = load_rec(v, i);
        const bool staged = ns >= 0 && !(r.mode & MODE_SORTED);
        // rows with the velocities of their points (ghosts: u_i)
        // (this lane's share of them)
        auto rows = [&](auto&& body) {
            if (staged) {
                for_rows_staged_sub<FIT_BATCH, LPP, true>(v, g, i, r, sub, sx, sy, sz,
                                                          [&](const double* a, double w,
                                                              const Pt* p) {
                    if (!p) {
                        body(a, w, p, 0.0, 0.0, 0.0);
                        return;
                    }
                    const int q = p->src;
                    body(a, w, p, su[q], sv[q], p->mirror ? -sw[q] : sw[q]);
                });
            } else {
                for_rows_sub<LPP>(v, g, i, r, sub, [&](const double* a, double w,
                                                       const Pt* p) {
                    double uj = 0.0, vj = 0.0, wj = 0.0;
                    if (p) point_velocity(v, *p, uj, vj, wj);
                    body(a, w, p, uj, vj, wj);
                });
            }
        };
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
            // (lane 0's share: every lane computes the closure)
            th[0] = lead ? mub * prm.I0 / den : 0.0;
            th[1] = lead ? mub * I / den : 0.0;
            th[2] = lead ? -mub * (prm.mu_2 - prm.mu_s) * I / (den * den) : 0.0;
        } else if (cl.branch == 2) {
            phib = Pb * prm.rho_s * prm.beta;
        }
        if (lead) B.a[6][i] += -phib / (V * V);
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
        // the moments of the rows, as the reverse pass 2 summed them
        double M[31];
#pragma unroll
        for (int q = 0; q < 31; ++q) M[q] = B.M[(int64_t)q * n + i];
        double U[45];
        gram_from_moments(M, U);
        const double ratio = lin ? cholesky<3>(U) : cholesky<9>(U);
        if (!(ratio > 0.0)) {
            if (lead) raise_error(B.err, ERR_NUMERIC, i);
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
            double au[3] = {0.0, 0.0, 0.0}, ax = 0.0, ay = 0.0, az = 0.0;
            rows([&](const double* a, double, const Pt* p, double uj, double vj,
                     double wj) {
                double b[3] = {0.0, 0.0, 0.0};   // ghosts carry u_i
                if (p) {
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
                au[0] -= bb[0];
                au[1] -= bb[1];
                au[2] -= bb[2];
                double gx, gy, gz;
                row_xi_bar(Ab, a[0], a[1], a[2], gx, gy, gz);
                gx *= ih;
                gy *= ih;
                gz *= ih;
                ax -= gx;
                ay -= gy;
                az -= gz;
                const double sg = p->mirror ? -1.0 : 1.0;
                const double cr[6] = {bb[0], bb[1], sg * bb[2], gx, gy, sg * gz};
                deliver(B, n, acc, staged, p->src, cr);
            });
            // this particle's own terms (other particles' rows arrive in
            // B.recv)
            if (LPP > 1) {
#pragma unroll
                for (int f = 0; f < 3; ++f) au[f] = lane_sum<LPP>(au[f]);
                ax = lane_sum<LPP>(ax);
                ay = lane_sum<LPP>(ay);
                az = lane_sum<LPP>(az);
            }
            if (lead) {
                B.a[3][i] += au[0];
                B.a[4][i] += au[1];
                B.a[5][i] += au[2];
                B.a[0][i] += ax;
                B.a[1][i] += ay;
                B.a[2][i] += az;
            }
        }
    }
    if (ns >= 0) {
        __syncthreads();
        acc_flush<NT>(B, v.n, acc, v.tile_src + tile * STAGE_CAP, ns);
    }
    // parameter cotangents: one atomic per block when the block lies in
    // one system, else one per thread (the staged rows are dead once every
    // thread has passed the first barrier)
    double (*red)[NT] = reinterpret_cast<double (*)[NT]>(lds);
    sys_t[t] = s;
    __syncthreads();
    const int s0 = sys_t[0];
    const bool uniform = __syncthreads_and((s == s0 || s < 0) ? 1 : 0) != 0 && s0 >= 0;
    if (uniform) {
        red[0][t] = th[0];
        red[1][t] = th[1];
        red[2][t] = th[2];
        __syncthreads();
        for (int w = NT / 2; w > 0; w >>= 1) {
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

// The fold of pass 1 (u, v, w, x, y, z received) written straight to the
// caller's order: adj_in[perm[j]] = acc[j] + received[j] (perm null:
// adj_in[j]).
__global__ void k_fold_unpermute(int64_t n, const int32_t* perm, AdjBufs B, Ptr7 out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t o = perm ? perm[j] : j;
    const double* r = B.recv;
    double v[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) v[a] = B.a[a][j];
    v[3] += r[j];
    v[4] += r[n + j];
    v[5] += r[2 * n + j];
    v[0] += r[3 * n + j];
    v[1] += r[4 * n + j];
    v[2] += r[5 * n + j];
#pragma unroll
    for (int a = 0; a < 7; ++a) const_cast<double*>(out.p[a])[o] = v[a];
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
    // contributions to other particles arrive in B.recv (6 x n), cleared
    // before each reverse pass and added to the accumulators after it
    hipStream_t s = c->stream;
    B.recv = w.adj_recv;
    B.M = w.adj_M;
    const int mo = c->map_ok ? 1 : 0;
    // (k_adj_init clears the receive buffers, the fold of pass 2 clears
    // them again for pass 1, whose fold writes the result)
    hipLaunchKernelGGL(k_adj_init, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, seed, B);
    hipLaunchKernelGGL(k_adj_pass2<ADJ_LPP>, dim3(blocks_for(n)), dim3(BLOCK * ADJ_LPP), 0, s,
                       v, seed, B, mo);
    hipLaunchKernelGGL(k_fold2, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, B);
    hipLaunchKernelGGL(k_adj_pass1<ADJ_LPP>, dim3(blocks_for(n)), dim3(BLOCK * ADJ_LPP), 0, s,
                       v, B, mo);
    hipLaunchKernelGGL(k_fold_unpermute, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, perm, B,
                       dout);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "adjoint launch");
    return LP_OK;
}

}  // namespace lp
