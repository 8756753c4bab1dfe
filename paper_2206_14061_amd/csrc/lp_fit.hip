// Least-squares derivatives (Sec. 3.1 step 7), mu(I) closure (Sec. 2.2,
// 2.2.1), right-hand side (Sec. 2.1) and explicit update (Sec. 3.1 steps
// 8 and 10).
//
// Fit: one thread per particle accumulates the 9x9 Gram matrix
// G = sum_r w a_r a_r^T and the moments sum_r w a_r b_r of its Taylor rows
// (stencil rows plus ghost rows), factors G = U^T U (Cholesky) and solves.
// The rows are scaled by 1/h, so G is well conditioned on every regular
// stencil (the pivot ratio min U_jj / max U_jj is checked); this needs no
// cross-lane reductions and keeps every accumulator in registers.  A
// stencil whose pivot ratio falls below the refit threshold is refitted
// by float64 Householder QR (a wavefront per stencil), which
// also applies the rank test min|r_jj|/max|r_jj| < fallback_tol.
//
// The second fit (P, eta) needs only first derivatives: pass 1 stores
// rows 0-2 of G^{-1}, so pass 2 costs two moment accumulations and a 3x9
// product per particle.
#include "lp_finish.h"

namespace lp {

namespace {

inline unsigned int blocks_for(int64_t n, int per = BLOCK)
{
    return (unsigned int)((n + per - 1) / per);
}

// ---- Householder QR for refits -----------------------------------------
//
// One wavefront refits one particle.  Stencil row k (k < MAXROWS) lives in
// lane k % 64, register slot k / 64.  The column norm and the dot products
// of each Householder step are wavefront sums (a xor butterfly leaves the
// same value in every lane, so every branch on them is uniform); R's rows
// and Q^T b are read by broadcast, and every lane back-substitutes (nine
// unknowns at most), so each lane ends with the same coefficients.

constexpr int QR_TPB = 256;     // four wavefronts per block, one refit each
constexpr int QR_BLOCKS = 256;  // 1,024 refits in flight

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) x += __shfl_xor(x, d);
    return x;
}

// Householder least squares of particle i's rows, called by all 64 lanes
// of a wavefront together.  vals(p, out) gives the nf (<= 8) field values
// at a stencil point (p != null) or at the ghosts (p == null); own: the
// values at the particle.  coef (nf x 9, ld 9) receives derivative
// estimates in every lane.  Returns FLAG_QR plus FLAG_LINEAR when the
// linear fallback (fewer than 9 rows, or the rank test
// min|r_jj| / max|r_jj| < fallback_tol) was taken.
template <class Vals>
__device__ uint8_t qr_fit_point(const View& v, const GridInfo& g, int64_t i,
                                const Rec& r, int nf, const double* own,
                                Vals&& vals, double* coef)
{
    static_assert(MAXROWS <= 128, "two rows per lane");
    const int lane = (int)(threadIdx.x & 63u);
    double A[2][9], B[2][8];
    auto build = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int q = 0; q < 9; ++q) A[h][q] = 0.0;
#pragma unroll
            for (int f = 0; f < 8; ++f) B[h][f] = 0.0;
        }
        int k = 0;
        return for_rows(v, g, i, r, [&](const double* a, double w, const Pt* p) {
            if (k >= MAXROWS) return;
            if ((k & 63) == lane) {
                const double sw = sqrt(w);
                double fj[8];
                vals(p, fj);
                const bool hi = k >= 64;
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const double x = sw * a[q];
                    A[0][q] = hi ? A[0][q] : x;
                    A[1][q] = hi ? x : A[1][q];
                }
#pragma unroll
                for (int f = 0; f < 8; ++f) {
                    if (f >= nf) break;
                    const double y = sw * (fj[f] - own[f]);
                    B[0][f] = hi ? B[0][f] : y;
                    B[1][f] = hi ? y : B[1][f];
                }
            }
            ++k;
        });
    };
    // QR of the first nc columns, applied to B; rd: the diagonal of R
    double rd[9];
    auto factor = [&](int nc) -> double {
        double rmin = INFINITY, rmax = 0.0;
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            if (j >= nc) break;
            const double x0 = lane >= j ? A[0][j] : 0.0, x1 = A[1][j];
            const double nrm = sqrt(wave_sum(x0 * x0 + x1 * x1));
            const double ajj = __shfl(A[0][j], j);
            if (nrm == 0.0) {
                rd[j] = 0.0;
                rmin = 0.0;
                continue;
            }
            const double alpha = ajj >= 0.0 ? -nrm : nrm;
            if (lane == j) A[0][j] = ajj - alpha;   // Householder vector in column j
            const double beta = 1.0 / (nrm * (nrm + fabs(ajj)));  // 2 / v^T v
            const double v0 = lane >= j ? A[0][j] : 0.0, v1 = A[1][j];
#pragma unroll
            for (int l = j + 1; l < 9; ++l) {
                if (l >= nc) break;
                const double f = beta * wave_sum(v0 * A[0][l] + v1 * A[1][l]);
                if (lane >= j) A[0][l] -= f * v0;
                A[1][l] -= f * v1;
            }
#pragma unroll
            for (int l = 0; l < 8; ++l) {
                if (l >= nf) break;
                const double f = beta * wave_sum(v0 * B[0][l] + v1 * B[1][l]);
                if (lane >= j) B[0][l] -= f * v0;
                B[1][l] -= f * v1;
            }
            rd[j] = alpha;
            rmin = fmin(rmin, fabs(alpha));
            rmax = fmax(rmax, fabs(alpha));
        }
        return rmax > 0.0 ? rmin / rmax : 0.0;
    };
    // R c = Q^T b per field (rows j < nc of R and Q^T b sit in lanes j)
    auto solve = [&](int nc) {
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            if (f >= nf) break;
            double cf[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) cf[q] = 0.0;
#pragma unroll
            for (int j = 8; j >= 0; --j) {
                if (j >= nc) continue;
                double t = __shfl(B[0][f], j);
#pragma unroll
                for (int q = j + 1; q < 9; ++q)
                    if (q < nc) t -= __shfl(A[0][q], j) * cf[q];
                cf[j] = rd[j] != 0.0 ? t / rd[j] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 9; ++q)
                coef[f * 9 + q] = cf[q] * (q < 3 ? g.inv_h : g.inv_h * g.inv_h);
        }
    };
    uint8_t flags = FLAG_QR;
    int mt = build();
    if (mt > MAXROWS) mt = MAXROWS;
    const bool quad = order_rows(v, r, mt) >= 9;
    const double ratio = quad ? factor(9) : 0.0;
    if (quad && ratio >= v.fallback_tol) {
        solve(9);
        return flags;
    }
    flags |= FLAG_LINEAR;
    if (mt >= 3) {
        build();
        factor(3);
        solve(3);
    } else {
        for (int q = 0; q < nf * 9; ++q) coef[q] = 0.0;
    }
    return flags;
}

// Solves the Gram system for nf right-hand sides; coefficients unscaled
// (per unit h).  Returns false when the stencil needs a QR refit.
template <int NF>
__device__ __forceinline__ bool gram_solve(double (&G)[45], const double (&B)[NF][9],
                                           int mt, double redo_ratio, bool force_qr,
                                           double (&c)[NF][9], double (&ginv3)[27],
                                           bool want_ginv, uint8_t& fl)
{
    if (mt < 9) {
        fl = FLAG_LINEAR;
        const double ratio = cholesky<3>(G);
        if (ratio < redo_ratio || force_qr) return false;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int q = 0; q < 9; ++q) c[f][q] = q < 3 ? B[f][q] : 0.0;
            chol_solve<3>(G, c[f]);
        }
        if (want_ginv) ginv_rows<3>(G, ginv3);
    } else {
        fl = 0;
        const double ratio = cholesky<9>(G);
        if (ratio < redo_ratio || force_qr) return false;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
#pragma unroll
            for (int q = 0; q < 9; ++q) c[f][q] = B[f][q];
            chol_solve<9>(G, c[f]);
        }
        if (want_ginv) ginv_rows<9>(G, ginv3);
    }
    return true;
}

// ---- lp_fit_derivs -------------------------------------------------------


template <int NF>
__global__ __launch_bounds__(BLOCK) void k_fit_generic(View v, GenericFields F,
                                                       double* coef, uint8_t* flags,
                                                       int32_t* redo,
                                                       unsigned int* redo_n,
                                                       int force_qr)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (i >= v.n) return;
    const int64_t n = v.n;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    const Rec r = load_rec(v, i);
    double fi[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) fi[f] = F.f[(int64_t)f * n + i];
    double M[31], B[NF][9];
#pragma unroll
    for (int q = 0; q < 31; ++q) M[q] = 0.0;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 9; ++q) B[f][q] = 0.0;
    const int mt = for_rows(v, g, i, r, [&](const double* a, double w, const Pt* p) {
        moments_add(M, a, w);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double fj;
            if (!p) fj = F.gzero[f] ? 0.0 : fi[f];
            else if (p->mirror) fj = (double)F.msign[f] * F.f[(int64_t)f * n + p->src];
            else fj = F.f[(int64_t)f * n + p->src];
            const double b = w * (fj - fi[f]);
#pragma unroll
            for (int q = 0; q < 9; ++q) B[f][q] += a[q] * b;
        }
    });
    double G[45], c[NF][9], ginv3[27];
    gram_from_moments(M, G);
    uint8_t fl;
    if (!gram_solve<NF>(G, B, order_rows(v, r, mt), v.redo_ratio, force_qr != 0, c, ginv3,
                        false, fl)) {
        redo[atomicAdd(redo_n, 1u)] = (int32_t)i;
        if (flags) flags[i] = FLAG_QR;
        return;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 9; ++q)
            coef[((int64_t)f * 9 + q) * n + i] =
                c[f][q] * (q < 3 ? g.inv_h : g.inv_h * g.inv_h);
    if (flags) flags[i] = fl;
}

__global__ __launch_bounds__(QR_TPB) void k_fit_generic_qr(
    View v, GenericFields F, double* coef, uint8_t* flags, const int32_t* redo,
    const unsigned int* redo_n, Counters* cnt)
{
    // a wavefront per refit
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const unsigned int total = *redo_n;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd(&cnt->qr_refits, (unsigned long long)total);
    const int64_t n = v.n;
    for (int64_t t = wave; t < (int64_t)total; t += nw) {
        const int64_t i = redo[t];
        const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
        const Rec r = load_rec(v, i);
        double own[8];
        for (int f = 0; f < F.k; ++f) own[f] = F.f[(int64_t)f * n + i];
        auto vals = [&](const Pt* p, double* out) {
            for (int f = 0; f < F.k; ++f) {
                if (!p) out[f] = F.gzero[f] ? 0.0 : own[f];
                else if (p->mirror) out[f] = (double)F.msign[f] * F.f[(int64_t)f * n + p->src];
                else out[f] = F.f[(int64_t)f * n + p->src];
            }
        };
        double c[8 * 9];
        const uint8_t fl = qr_fit_point(v, g, i, r, F.k, own, vals, c);
        if (lane == 0) {
            for (int f = 0; f < F.k; ++f)
                for (int q = 0; q < 9; ++q) coef[((int64_t)f * 9 + q) * n + i] = c[f * 9 + q];
            if (flags) flags[i] = fl;
        }
    }
}

// ---- lp_step pass 1: fit u, v, w + closure --------------------------------

// Factor, solve and store one particle's pass-1 fit from its Gram moments
// M and right-hand sides B (mt rows): coefficients, closure and the rows of
// G^-1 for pass 2, or a queued QR refit when the Gram matrix is too ill
// conditioned.  Only the lead lane of the particle writes.
__device__ __forceinline__ void pass1_solve(const View& v, const StepOut& o,
                                            const GridInfo& g, int s, int64_t i,
                                            const double (&M)[31], double (&B)[3][9],
                                            int mt, bool lead, int32_t* redo,
                                            unsigned int* redo_n, int force_qr)
{
    double G[45], c3[3][9], none[27];
    gram_from_moments(M, G);
    uint8_t fl;
    if (!gram_solve<3>(G, B, mt, v.redo_ratio, force_qr != 0, c3, none, false, fl)) {
        if (lead) {
            redo[atomicAdd(redo_n, 1u)] = (int32_t)i;
            o.flags[i] = FLAG_QR;
        }
        return;
    }
    if (!lead) return;
    double c[27];
#pragma unroll
    for (int q = 0; q < 27; ++q)
        c[q] = c3[q / 9][q % 9] * ((q % 9) < 3 ? g.inv_h : g.inv_h * g.inv_h);
    finish_pass1(v, v.prm[s], i, c, none, false, fl, o);
    if (mt < 9) store_ginv_rows<3>(G, o.hand, v.n, i);
    else store_ginv_rows<9>(G, o.hand, v.n, i);
}

// LPP lanes per particle: each lane accumulates every LPP-th row; the
// moments are summed across the lanes, every lane solves, lane 0 stores.
// With idx (a stencil size class): thread group t takes particle idx[t]
// for t < *icnt.
template <int LPP>
__global__ __launch_bounds__(BLOCK, 2) void k_pass1(View v, StepOut o,
                                                    int32_t* redo,
                                                    unsigned int* redo_n,
                                                    int force_qr, const int32_t* idx,
                                                    const uint32_t* icnt)
{
    const int64_t gt = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    int64_t i = gt / LPP;
    const int sub = (int)(gt % LPP);
    if (idx) {
        if (i >= (int64_t)*icnt) return;
        i = idx[i];
    }
    if (i >= v.n) return;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const Rec r = load_rec(v, i);
    const double ui = v.u[i], vi = v.v[i], wi = v.w[i];
    double M[31], B[3][9];
#pragma unroll
    for (int q = 0; q < 31; ++q) M[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) B[0][q] = B[1][q] = B[2][q] = 0.0;
    int mt = for_rows_sub<LPP>(v, g, i, r, sub, [&](const double* a, double w,
                                                    const Pt* p) {
        moments_add(M, a, w);
        if (!p) return;   // ghosts carry u_i (b = 0)
        double uj, vj, wj;
        point_velocity(v, *p, uj, vj, wj);
        const double b0 = w * (uj - ui), b1 = w * (vj - vi), b2 = w * (wj - wi);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            B[0][q] += a[q] * b0;
            B[1][q] += a[q] * b1;
            B[2][q] += a[q] * b2;
        }
    });
    if (LPP > 1) {
        mt = lane_sum<LPP>(mt);
#pragma unroll
        for (int q = 0; q < 31; ++q) M[q] = lane_sum<LPP>(M[q]);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            B[0][q] = lane_sum<LPP>(B[0][q]);
            B[1][q] = lane_sum<LPP>(B[1][q]);
            B[2][q] = lane_sum<LPP>(B[2][q]);
        }
    }
    pass1_solve(v, o, g, s, i, M, B, order_rows(v, r, mt), sub == 0, redo, redo_n,
                force_qr);
}

// Pass 1 with the neighbours of the block's tile staged in LDS (one lane
// per particle): the positions and velocities of the tile's list sources
// are loaded once, coalesced, and every stencil row reads them from LDS.
// A tile that is not staged, and a particle on the sorted path, read their
// neighbours from global memory as k_pass1<1> does, and so does every
// tile when the tile map is stale (map_ok = 0).  UNIT: the weights are unit
// (known at compile time).
template <bool UNIT>
// skip_rows > 0: particles whose stencils have at most skip_rows rows
// (ghosts included) are left to the size-class launches.
__global__ __launch_bounds__(BLOCK, 2) void k_pass1_st(View v, StepOut o,
                                                       int32_t* redo,
                                                       unsigned int* redo_n,
                                                       int force_qr, int map_ok,
                                                       int skip_rows)
{
    __shared__ double sx[STAGE_CAP], sy[STAGE_CAP], sz[STAGE_CAP];
    __shared__ double su[STAGE_CAP], sv[STAGE_CAP], sw[STAGE_CAP];
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = tile * BLOCK + threadIdx.x;
    const int tc = map_ok ? v.tile_cnt[tile] : -1;
    const int S = tc <= STAGE_CAP ? tc : -1;   // -1: not staged
    if (S >= 0) {
        stage_pass1(v, tile, S, sx, sy, sz, su, sv, sw);
        __syncthreads();
    }
    if (i >= v.n) return;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const Rec r = load_rec(v, i);
    if (skip_rows > 0 && r.m + __popc((unsigned)r.gm & 0xFFu) <= skip_rows) return;
    const double ui = v.u[i], vi = v.v[i], wi = v.w[i];
    double M[31], B[3][9];
#pragma unroll
    for (int q = 0; q < 31; ++q) M[q] = 0.0;
#pragma unroll
    for (int q = 0; q < 9; ++q) B[0][q] = B[1][q] = B[2][q] = 0.0;
    auto add_b = [&](const double* a, double w, double uj, double vj, double wj) {
        const double b0 = w * (uj - ui), b1 = w * (vj - vi), b2 = w * (wj - wi);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            B[0][q] += a[q] * b0;
            B[1][q] += a[q] * b1;
            B[2][q] += a[q] * b2;
        }
    };
    int mt;
    if (S >= 0 && !(r.mode & MODE_SORTED)) {
        mt = for_rows_staged<FIT_BATCH, UNIT>(v, g, i, r, sx, sy, sz,
                                        [&](const double* a, double w, const Pt* p) {
            moments_add(M, a, w);
            if (!p) return;   // ghosts carry u_i (b = 0)
            const int q = p->src;
            add_b(a, w, su[q], sv[q], p->mirror ? -sw[q] : sw[q]);
        });
    } else {
        mt = for_rows(v, g, i, r, [&](const double* a, double w, const Pt* p) {
            moments_add(M, a, w);
            if (!p) return;
            double uj, vj, wj;
            point_velocity(v, *p, uj, vj, wj);
            add_b(a, w, uj, vj, wj);
        });
    }
    pass1_solve(v, o, g, s, i, M, B, order_rows(v, r, mt), true, redo, redo_n, force_qr);
}

__global__ __launch_bounds__(QR_TPB) void k_pass1_qr(View v, StepOut o,
                                                    const int32_t* redo,
                                                    const unsigned int* redo_n,
                                                    Counters* cnt)
{
    // a wavefront per refit
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const unsigned int total = *redo_n;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd(&cnt->qr_refits, (unsigned long long)total);
    for (int64_t t = wave; t < (int64_t)total; t += nw) {
        const int64_t i = redo[t];
        const int s = sys_of(v.off, v.n_sys, i);
        const GridInfo& g = v.grid[s];
        const Rec r = load_rec(v, i);
        const double own[3] = {v.u[i], v.v[i], v.w[i]};
        auto vals = [&](const Pt* p, double* out) {
            if (!p) {
                out[0] = own[0]; out[1] = own[1]; out[2] = own[2];
            } else {
                point_velocity(v, *p, out[0], out[1], out[2]);
            }
        };
        double c[27], none[27];
        const uint8_t fl = qr_fit_point(v, g, i, r, 3, own, vals, c);
        if (lane == 0) finish_pass1(v, v.prm[s], i, c, none, false, fl, o);
    }
}

// lp_rheology_rhs: closure from given coefficients, Gram factor for pass 2
__global__ __launch_bounds__(BLOCK) void k_closure_coef(View v, const double* coef_u,
                                                        StepOut o, int32_t* redo,
                                                        unsigned int* redo_n,
                                                        int force_qr)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (i >= v.n) return;
    const int64_t n = v.n;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const Rec r = load_rec(v, i);
    double c[27];
#pragma unroll
    for (int q = 0; q < 27; ++q) c[q] = coef_u[(int64_t)q * n + i];
    double M[31], G[45];
#pragma unroll
    for (int q = 0; q < 31; ++q) M[q] = 0.0;
    const int mt = for_rows(v, g, i, r, [&](const double* a, double w, const Pt*) {
        moments_add(M, a, w);
    });
    gram_from_moments(M, G);
    const double B[1][9] = {{0, 0, 0, 0, 0, 0, 0, 0, 0}};
    double c1[1][9], ginv3[27];
    uint8_t fl;
    const bool ok = gram_solve<1>(G, B, order_rows(v, r, mt), v.redo_ratio, force_qr != 0,
                                  c1, ginv3, true, fl);
    if (!ok) {
        redo[atomicAdd(redo_n, 1u)] = (int32_t)i;
        fl = FLAG_QR;
    }
    finish_pass1(v, v.prm[s], i, c, ginv3, ok, fl, o);
}

// ---- pass 2: fit of P and eta, right-hand side, update --------------------

// Gradients of P and eta from the pass-2 right-hand sides (the stored rows
// of G^-1), then the right-hand side and update of particle i.
__device__ __forceinline__ void pass2_finish(const View& v, const lp_params& prm,
                                             const GridInfo& g, int64_t i,
                                             const double* hand, const double (&yP)[9],
                                             const double (&yE)[9], double Ei,
                                             const RhsOut& o)
{
    const int64_t n = v.n;
    double gP[3], gE[3];
#pragma unroll
    for (int rr = 0; rr < 3; ++rr) {
        double sp = 0.0, se = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const double gi = hand[(int64_t)(rr * 9 + q) * n + i];
            sp += gi * yP[q];
            se += gi * yE[q];
        }
        gP[rr] = sp * g.inv_h;
        gE[rr] = se * g.inv_h;
    }
    double hv[11];
    load_hand_tail(hand, n, i, Ei, hv);
    finish_rhs(v, prm, i, hv, gP, gE, o);
}

#ifndef LP_PASS2_BATCH
#define LP_PASS2_BATCH 8
#endif
// Stencil rows the pass-2 fit loads together: its accumulators are few,
// so a deeper batch than pass 1's still fits in registers.
constexpr int PASS2_BATCH = LP_PASS2_BATCH;

template <int LPP>
__global__ __launch_bounds__(BLOCK) void k_pass2(View v, const double* P,
                                                 const double* eta,
                                                 const double* hand,
                                                 const uint8_t* flags, RhsOut o,
                                                 const int32_t* idx, const uint32_t* icnt)
{
    const int64_t gt = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    int64_t i = gt / LPP;
    const int sub = (int)(gt % LPP);
    if (idx) {
        if (i >= (int64_t)*icnt) return;
        i = idx[i];
    }
    if (i >= v.n) return;
    if (flags[i] & FLAG_QR) return;
    const int64_t n = v.n;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const lp_params& prm = v.prm[s];
    const Rec r = load_rec(v, i);
    const double Pi = P[i], Ei = eta[i];
    double yP[9], yE[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) yP[q] = yE[q] = 0.0;
    for_rows_sub<LPP, PASS2_BATCH>(v, g, i, r, sub, [&](const double* a, double w,
                                                         const Pt* p) {
        double Pj, Ej;
        pass2_values(v, P, eta, p, prm, Pj, Ej);
        const double bP = w * (Pj - Pi), bE = w * (Ej - Ei);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            yP[q] += a[q] * bP;
            yE[q] += a[q] * bE;
        }
    });
    if (LPP > 1) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            yP[q] = lane_sum<LPP>(yP[q]);
            yE[q] = lane_sum<LPP>(yE[q]);
        }
    }
    if (sub != 0) return;
    pass2_finish(v, prm, g, i, hand, yP, yE, Ei, o);
}

// Pass 2 with the neighbours of the block's tile staged in LDS (one lane
// per particle): positions, P, eta and the pressure a mirror of each list
// source carries are loaded once, coalesced, and every stencil row reads
// them from LDS.  A tile that is not staged, and a particle on the sorted
// path, read their neighbours from global memory as k_pass2<1> does, and
// so does every tile when the tile map is stale (map_ok = 0).  UNIT: the
// weights are unit (known at compile time).
template <bool UNIT>
__global__ __launch_bounds__(BLOCK) void k_pass2_st(View v, const double* P,
                                                    const double* eta,
                                                    const double* hand,
                                                    const uint8_t* flags, RhsOut o,
                                                    int map_ok, int skip_rows)
{
    __shared__ double sx[STAGE_CAP], sy[STAGE_CAP], sz[STAGE_CAP];
    __shared__ double sP[STAGE_CAP], sE[STAGE_CAP], sM[STAGE_CAP];
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = tile * BLOCK + threadIdx.x;
    const int tc = map_ok ? v.tile_cnt[tile] : -1;
    const int S = tc <= STAGE_CAP ? tc : -1;   // -1: not staged
    if (S >= 0) {
        stage_pass2(v, P, eta, tile, S, sx, sy, sz, sP, sE, sM);
        __syncthreads();
    }
    if (i >= v.n) return;
    if (flags[i] & FLAG_QR) return;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const lp_params& prm = v.prm[s];
    const Rec r = load_rec(v, i);
    if (skip_rows > 0 && r.m + __popc((unsigned)r.gm & 0xFFu) <= skip_rows) return;
    const double Pi = P[i], Ei = eta[i];
    double yP[9], yE[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) yP[q] = yE[q] = 0.0;
    auto add_y = [&](const double* a, double w, double Pj, double Ej) {
        const double bP = w * (Pj - Pi), bE = w * (Ej - Ei);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            yP[q] += a[q] * bP;
            yE[q] += a[q] * bE;
        }
    };
    if (S >= 0 && !(r.mode & MODE_SORTED)) {
        for_rows_staged<PASS2_BATCH, UNIT>(v, g, i, r, sx, sy, sz,
                                     [&](const double* a, double w, const Pt* p) {
            if (!p) add_y(a, w, 0.0, 0.0);
            else if (p->mirror) add_y(a, w, sM[p->src], 0.0);
            else add_y(a, w, sP[p->src], sE[p->src]);
        });
    } else {
        for_rows<PASS2_BATCH>(v, g, i, r, [&](const double* a, double w, const Pt* p) {
            double Pj, Ej;
            pass2_values(v, P, eta, p, prm, Pj, Ej);
            add_y(a, w, Pj, Ej);
        });
    }
    pass2_finish(v, prm, g, i, hand, yP, yE, Ei, o);
}

// ---- refined FP32 fits ----------------------------------------------------
//
// The Gram moments and right-hand sides are accumulated and factored in
// float32; one sweep then forms the float64 residual r = b - A c of every
// row and corrects c by the float32 factor applied to A^T r.  The factor
// (45 floats) is kept for pass 2, which refines the same way.  A stencil
// whose float32 pivot ratio falls below the refit threshold takes the
// float64 Householder refit of the float64 path.

// rows per batch (measured at the 524,288-particle column): the moment
// sweeps take those of the float64 fits; pass 1's float64 residual sweep,
// which also holds three fields' coefficients and corrections, takes 2,
// pass 2's (two fields) 4
template <int B>
struct RowBatch {
    static constexpr int value = B;
};
constexpr int REF1_SWEEP_BATCH = 2;
constexpr int REF2_SWEEP_BATCH = 4;

template <int N>
__device__ __forceinline__ void store_factor(const float (&U)[45], float* uf, int64_t n,
                                             int64_t i)
{
#pragma unroll
    for (int q = 0; q < 45; ++q) uf[(int64_t)q * n + i] = U[q];
}

__device__ __forceinline__ void load_factor(float (&U)[45], const float* uf, int64_t n,
                                            int64_t i)
{
#pragma unroll
    for (int q = 0; q < 45; ++q) U[q] = uf[(int64_t)q * n + i];
}

// c += U^-1 U^-T d (the correction step), d in float64, solved in float32
template <int N, int NF>
__device__ __forceinline__ void refine_step(const float (&U)[45], const double (&d)[NF][9],
                                            double (&c)[NF][9])
{
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        float e[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) e[q] = q < N ? (float)d[f][q] : 0.0f;
        chol_solve<N>(U, e);
#pragma unroll
        for (int q = 0; q < N; ++q) c[f][q] += (double)e[q];
    }
}

// Both sweeps read their rows from the tile's LDS stage when the tile is
// staged (as k_pass1_st does), else from global memory.  UNIT: the
// weights are unit (known at compile time).
template <bool UNIT>
__global__ __launch_bounds__(BLOCK, 2) void k_pass1_ref(View v, StepOut o, float* uf,
                                                        int32_t* redo,
                                                        unsigned int* redo_n, int map_ok)
{
    __shared__ double sx[STAGE_CAP], sy[STAGE_CAP], sz[STAGE_CAP];
    __shared__ double su[STAGE_CAP], sv[STAGE_CAP], sw[STAGE_CAP];
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = tile * BLOCK + threadIdx.x;
    const int tc = map_ok ? v.tile_cnt[tile] : -1;
    const int S = tc <= STAGE_CAP ? tc : -1;   // -1: not staged
    if (S >= 0) {
        stage_pass1(v, tile, S, sx, sy, sz, su, sv, sw);
        __syncthreads();
    }
    if (i >= v.n) return;
    const int64_t n = v.n;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const Rec r = load_rec(v, i);
    const double ui = v.u[i], vi = v.v[i], wi = v.w[i];
    const bool staged = S >= 0 && !(r.mode & MODE_SORTED);
    // body(a, w, has, uj, vj, wj) for every row, bt.value rows at a time:
    // has is false for a ghost row, which carries u_i
    auto rows = [&](auto bt, auto&& body) -> int {
        constexpr int RB = decltype(bt)::value;
        if (staged)
            return for_rows_staged<RB, UNIT>(v, g, i, r, sx, sy, sz,
                                            [&](const double* a, double w, const Pt* p) {
                if (!p) {
                    body(a, w, false, ui, vi, wi);
                    return;
                }
                const int q = p->src;
                body(a, w, true, su[q], sv[q], p->mirror ? -sw[q] : sw[q]);
            });
        return for_rows<RB>(v, g, i, r, [&](const double* a, double w, const Pt* p) {
            double uj = ui, vj = vi, wj = wi;
            if (p) point_velocity(v, *p, uj, vj, wj);
            body(a, w, p != nullptr, uj, vj, wj);
        });
    };
    // ---- float32 moments and right-hand sides
    float M[31], B[3][9];
#pragma unroll
    for (int q = 0; q < 31; ++q) M[q] = 0.0f;
#pragma unroll
    for (int q = 0; q < 9; ++q) B[0][q] = B[1][q] = B[2][q] = 0.0f;
    const int mt = rows(RowBatch<FIT_BATCH>{}, [&](const double* a, double w, bool has,
                                                   double uj, double vj, double wj) {
        float af[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) af[q] = (float)a[q];
        moments_add(M, af, (float)w);
        if (!has) return;
        const float b0 = (float)(w * (uj - ui)), b1 = (float)(w * (vj - vi)),
                    b2 = (float)(w * (wj - wi));
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            B[0][q] += af[q] * b0;
            B[1][q] += af[q] * b1;
            B[2][q] += af[q] * b2;
        }
    });
    float U[45];
    gram_from_moments(M, U);
    const bool lin = order_rows(v, r, mt) < 9;
    const float ratio = lin ? cholesky<3>(U) : cholesky<9>(U);
    // one float32 correction step needs a better conditioned factor than
    // the float64 path: four times the pivot-ratio threshold
    if (!(ratio >= 4.0f * (float)v.redo_ratio)) {
        redo[atomicAdd(redo_n, 1u)] = (int32_t)i;
        o.flags[i] = FLAG_QR;
        return;
    }
    // the float32 solution; the residual sweep widens it exactly to float64
    float cf[3][9];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        float e[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) e[q] = (lin && q >= 3) ? 0.0f : B[f][q];
        if (lin) chol_solve<3>(U, e);
        else chol_solve<9>(U, e);
#pragma unroll
        for (int q = 0; q < 9; ++q) cf[f][q] = (lin && q >= 3) ? 0.0f : e[q];
    }
    // the factor goes to memory: pass 2 needs it, and it is dead here
    // until the correction
    if (lin) store_factor<3>(U, uf, n, i);
    else store_factor<9>(U, uf, n, i);
    // ---- float64 residual sweep: d = A^T W (b - A c)
    double d[3][9];
#pragma unroll
    for (int q = 0; q < 9; ++q) d[0][q] = d[1][q] = d[2][q] = 0.0;
    rows(RowBatch<REF1_SWEEP_BATCH>{}, [&](const double* a, double w, bool has, double uj,
                                           double vj, double wj) {
        double b0 = 0.0, b1 = 0.0, b2 = 0.0;   // ghosts carry u_i
        if (has) {
            b0 = uj - ui;
            b1 = vj - vi;
            b2 = wj - wi;
        }
        double r0 = b0, r1 = b1, r2 = b2;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            r0 -= a[q] * (double)cf[0][q];
            r1 -= a[q] * (double)cf[1][q];
            r2 -= a[q] * (double)cf[2][q];
        }
        r0 *= w;
        r1 *= w;
        r2 *= w;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            d[0][q] += a[q] * r0;
            d[1][q] += a[q] * r1;
            d[2][q] += a[q] * r2;
        }
    });
    load_factor(U, uf, n, i);
    double c[3][9];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int q = 0; q < 9; ++q) c[f][q] = (double)cf[f][q];
    if (lin) refine_step<3, 3>(U, d, c);
    else refine_step<9, 3>(U, d, c);
    double cs[27];
#pragma unroll
    for (int q = 0; q < 27; ++q)
        cs[q] = c[q / 9][q % 9] * ((q % 9) < 3 ? g.inv_h : g.inv_h * g.inv_h);
    const double none[27] = {};
    finish_pass1(v, v.prm[s], i, cs, none, false, lin ? FLAG_LINEAR : 0, o);
}

// Both sweeps read their rows from the tile's LDS stage when the tile is
// staged (as k_pass2_st does), else from global memory.
template <bool UNIT>
__global__ __launch_bounds__(BLOCK, 2) void k_pass2_ref(View v, const double* P,
                                                     const double* eta,
                                                     const double* hand,
                                                     const float* uf,
                                                     const uint8_t* flags, RhsOut o,
                                                     int map_ok)
{
    __shared__ double sx[STAGE_CAP], sy[STAGE_CAP], sz[STAGE_CAP];
    __shared__ double sP[STAGE_CAP], sE[STAGE_CAP], sM[STAGE_CAP];
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const int64_t i = tile * BLOCK + threadIdx.x;
    const int tc = map_ok ? v.tile_cnt[tile] : -1;
    const int S = tc <= STAGE_CAP ? tc : -1;   // -1: not staged
    if (S >= 0) {
        stage_pass2(v, P, eta, tile, S, sx, sy, sz, sP, sE, sM);
        __syncthreads();
    }
    if (i >= v.n) return;
    const uint8_t fl = flags[i];
    if (fl & FLAG_QR) return;
    const int64_t n = v.n;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const lp_params& prm = v.prm[s];
    const Rec r = load_rec(v, i);
    const bool lin = fl & FLAG_LINEAR;
    const double Pi = P[i], Ei = eta[i];
    const bool staged = S >= 0 && !(r.mode & MODE_SORTED);
    // body(a, w, Pj, Ej) for every row (what pass2_values gives), bt.value
    // rows at a time
    auto rows = [&](auto bt, auto&& body) {
        constexpr int RB = decltype(bt)::value;
        if (staged)
            for_rows_staged<RB, UNIT>(v, g, i, r, sx, sy, sz,
                                             [&](const double* a, double w, const Pt* p) {
                if (!p) body(a, w, 0.0, 0.0);
                else if (p->mirror) body(a, w, sM[p->src], 0.0);
                else body(a, w, sP[p->src], sE[p->src]);
            });
        else
            for_rows<RB>(v, g, i, r, [&](const double* a, double w, const Pt* p) {
                double Pj, Ej;
                pass2_values(v, P, eta, p, prm, Pj, Ej);
                body(a, w, Pj, Ej);
            });
    };
    // ---- float32 right-hand sides and solve
    float yP[9], yE[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) yP[q] = yE[q] = 0.0f;
    rows(RowBatch<PASS2_BATCH>{}, [&](const double* a, double w, double Pj, double Ej) {
        const float bP = (float)(w * (Pj - Pi)), bE = (float)(w * (Ej - Ei));
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const float aq = (float)a[q];
            yP[q] += aq * bP;
            yE[q] += aq * bE;
        }
    });
    float U[45];
    load_factor(U, uf, n, i);
    double c[2][9];
    {
        float e0[9], e1[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            e0[q] = (lin && q >= 3) ? 0.0f : yP[q];
            e1[q] = (lin && q >= 3) ? 0.0f : yE[q];
        }
        if (lin) {
            chol_solve<3>(U, e0);
            chol_solve<3>(U, e1);
        } else {
            chol_solve<9>(U, e0);
            chol_solve<9>(U, e1);
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            c[0][q] = (lin && q >= 3) ? 0.0 : (double)e0[q];
            c[1][q] = (lin && q >= 3) ? 0.0 : (double)e1[q];
        }
    }
    // ---- float64 residual sweep and correction
    double d[2][9];
#pragma unroll
    for (int q = 0; q < 9; ++q) d[0][q] = d[1][q] = 0.0;
    rows(RowBatch<REF2_SWEEP_BATCH>{}, [&](const double* a, double w, double Pj, double Ej) {
        double rP = Pj - Pi, rE = Ej - Ei;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            rP -= a[q] * c[0][q];
            rE -= a[q] * c[1][q];
        }
        rP *= w;
        rE *= w;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            d[0][q] += a[q] * rP;
            d[1][q] += a[q] * rE;
        }
    });
    if (lin) refine_step<3, 2>(U, d, c);
    else refine_step<9, 2>(U, d, c);
    double gP[3], gE[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        gP[q] = c[0][q] * g.inv_h;
        gE[q] = c[1][q] * g.inv_h;
    }
    double hv[11];
    load_hand_tail(hand, n, i, Ei, hv);
    finish_rhs(v, prm, i, hv, gP, gE, o);
}

__global__ __launch_bounds__(QR_TPB) void k_pass2_qr(View v, const double* P,
                                                    const double* eta,
                                                    const double* hand,
                                                    const int32_t* redo,
                                                    const unsigned int* redo_n,
                                                    RhsOut o)
{
    // a wavefront per refit
    const int lane = (int)(threadIdx.x & 63u);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    const unsigned int total = *redo_n;
    const int64_t n = v.n;
    for (int64_t t = wave; t < (int64_t)total; t += nw) {
        const int64_t i = redo[t];
        const int s = sys_of(v.off, v.n_sys, i);
        const GridInfo& g = v.grid[s];
        const lp_params& prm = v.prm[s];
        const Rec r = load_rec(v, i);
        const double own[2] = {P[i], eta[i]};
        auto vals = [&](const Pt* p, double* out) {
            pass2_values(v, P, eta, p, prm, out[0], out[1]);
        };
        double c[18];
        const uint8_t fl = qr_fit_point(v, g, i, r, 2, own, vals, c);
        if (lane == 0) {
            if (o.flags)
                o.flags[i] = (uint8_t)((o.flags[i] & ~FLAG_LINEAR) | (fl & FLAG_LINEAR) | FLAG_QR);
            const double gP[3] = {c[0], c[1], c[2]};
            const double gE[3] = {c[9], c[10], c[11]};
            double hv[11];
            load_hand_tail(hand, n, i, eta[i], hv);
            finish_rhs(v, prm, i, hv, gP, gE, o);
        }
    }
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

// Clears the fits' refit counter unless the stencil build enqueued last
// has (k_mirror_count clears it with the step's other counters).
void redo_reset(lp_ctx* c)
{
    if (!c->redo_clear)
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, c->stream, c->w.redo_n);
    c->redo_clear = false;
}

__global__ void k_zero_classes(uint32_t* cnt)
{
    if (threadIdx.x < NCLASS) cnt[threadIdx.x] = 0u;
}

// Sorts the real particles into stencil size classes by their rows (kept
// stencil rows plus ghost rows): class 0 at most CLASS_ROWS0, class 1 at
// most CLASS_ROWS1, class 2 more.  Appends are wave-aggregated; the order
// inside a class is immaterial (every particle's fit is its own).
__global__ __launch_bounds__(BLOCK) void k_classify(View v, int32_t* idx, uint32_t* cnt)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t n = v.n;
    int cls = -1;
    if (i < n) {
        const int m = v.rec[REC_M * n + i] + __popc((unsigned)v.rec[REC_GM * n + i] & 0xFFu);
        cls = m <= CLASS_ROWS0 ? 0 : (m <= CLASS_ROWS1 ? 1 : 2);
    }
    const int lane = (int)(threadIdx.x & 63u);
#pragma unroll
    for (int c = 0; c < NCLASS; ++c) {
        const unsigned long long mask = __ballot(cls == c);
        if (!mask) continue;
        const int leader = __ffsll(mask) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(&cnt[c], (uint32_t)__popcll(mask));
        base = __shfl(base, leader);
        if (cls == c)
            idx[(int64_t)c * n + base + __popcll(mask & ((1ull << lane) - 1ull))] = (int32_t)i;
    }
}

__global__ void k_copy_u8(int64_t n, const uint8_t* a, uint8_t* b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

}  // namespace

static lp_status need_stencils(lp_ctx* c)
{
    if (!c->stencils_ok) {
        c->err = "lp_neighbors (or lp_step) must build the stencils first";
        return LP_E_STATE;
    }
    return LP_OK;
}

namespace {

void launch_pass1(lp_ctx* c, int lpp, const View& v, const StepOut& so, int fq)
{
    Work& w = c->w;
    const int64_t n = c->n;
    const int32_t* no = nullptr;
    const uint32_t* nc = nullptr;
    switch (lpp) {
    case 4:
        hipLaunchKernelGGL((k_pass1<4>), dim3(blocks_for(4 * n)), dim3(BLOCK), 0,
                           c->stream, v, so, w.redo, w.redo_n, fq, no, nc);
        break;
    case 2:
        hipLaunchKernelGGL((k_pass1<2>), dim3(blocks_for(2 * n)), dim3(BLOCK), 0,
                           c->stream, v, so, w.redo, w.redo_n, fq, no, nc);
        break;
    default:
        if (c->cfg.weight == LP_W_UNIT)
            hipLaunchKernelGGL(k_pass1_st<true>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, so, w.redo, w.redo_n, fq, c->map_ok ? 1 : 0,
                               0);
        else
            hipLaunchKernelGGL(k_pass1_st<false>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, so, w.redo, w.redo_n, fq, c->map_ok ? 1 : 0,
                               0);
    }
}

void launch_pass2(lp_ctx* c, int lpp, const View& v, const RhsOut& o)
{
    Work& w = c->w;
    const int64_t n = c->n;
    const double* P = w.P;
    const double* E = w.eta;
    const double* H = w.hand;
    const uint8_t* F = w.flags;
    const int32_t* no = nullptr;
    const uint32_t* nc = nullptr;
    switch (lpp) {
    case 4:
        hipLaunchKernelGGL((k_pass2<4>), dim3(blocks_for(4 * n)), dim3(BLOCK), 0,
                           c->stream, v, P, E, H, F, o, no, nc);
        break;
    case 2:
        hipLaunchKernelGGL((k_pass2<2>), dim3(blocks_for(2 * n)), dim3(BLOCK), 0,
                           c->stream, v, P, E, H, F, o, no, nc);
        break;
    default:
        if (c->cfg.weight == LP_W_UNIT)
            hipLaunchKernelGGL(k_pass2_st<true>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, P, E, H, F, o, c->map_ok ? 1 : 0, 0);
        else
            hipLaunchKernelGGL(k_pass2_st<false>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, P, E, H, F, o, c->map_ok ? 1 : 0, 0);
    }
}

// The size classes of the current stencils (one classification per
// stencil build, shared by both fits).
void classify(lp_ctx* c, const View& v)
{
    Work& w = c->w;
    hipLaunchKernelGGL(k_zero_classes, dim3(1), dim3(64), 0, c->stream, w.cls_cnt);
    if (c->n > 0)
        hipLaunchKernelGGL(k_classify, dim3(blocks_for(c->n)), dim3(BLOCK), 0, c->stream,
                           v, w.cls_idx, w.cls_cnt);
}

// One class of the pass-1 fit with lpp lanes per particle (the grid covers
// every particle; threads past the class's count return at once).
void launch_pass1_class(lp_ctx* c, int cls, int lpp, const View& v, const StepOut& so,
                        int fq)
{
    Work& w = c->w;
    const int64_t n = c->n;
    const int32_t* idx = w.cls_idx + (int64_t)cls * n;
    const uint32_t* cnt = w.cls_cnt + cls;
    if (lpp == 0) {
        // the largest class through the LDS-staged tile kernel
        const int mo = c->map_ok ? 1 : 0;
        if (c->cfg.weight == LP_W_UNIT)
            hipLaunchKernelGGL(k_pass1_st<true>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, so, w.redo, w.redo_n, fq, mo, CLASS_ROWS1);
        else
            hipLaunchKernelGGL(k_pass1_st<false>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, so, w.redo, w.redo_n, fq, mo, CLASS_ROWS1);
        return;
    }
    switch (lpp) {
    case 4:
        hipLaunchKernelGGL((k_pass1<4>), dim3(blocks_for(4 * n)), dim3(BLOCK), 0,
                           c->stream, v, so, w.redo, w.redo_n, fq, idx, cnt);
        break;
    case 2:
        hipLaunchKernelGGL((k_pass1<2>), dim3(blocks_for(2 * n)), dim3(BLOCK), 0,
                           c->stream, v, so, w.redo, w.redo_n, fq, idx, cnt);
        break;
    default:
        hipLaunchKernelGGL((k_pass1<1>), dim3(blocks_for(n)), dim3(BLOCK), 0,
                           c->stream, v, so, w.redo, w.redo_n, fq, idx, cnt);
    }
}

void launch_pass2_class(lp_ctx* c, int cls, int lpp, const View& v, const RhsOut& o)
{
    Work& w = c->w;
    const int64_t n = c->n;
    const int32_t* idx = w.cls_idx + (int64_t)cls * n;
    const uint32_t* cnt = w.cls_cnt + cls;
    const double* P = w.P;
    const double* E = w.eta;
    const double* H = w.hand;
    const uint8_t* F = w.flags;
    if (lpp == 0) {
        const int mo = c->map_ok ? 1 : 0;
        if (c->cfg.weight == LP_W_UNIT)
            hipLaunchKernelGGL(k_pass2_st<true>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, P, E, H, F, o, mo, CLASS_ROWS1);
        else
            hipLaunchKernelGGL(k_pass2_st<false>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, v, P, E, H, F, o, mo, CLASS_ROWS1);
        return;
    }
    switch (lpp) {
    case 4:
        hipLaunchKernelGGL((k_pass2<4>), dim3(blocks_for(4 * n)), dim3(BLOCK), 0,
                           c->stream, v, P, E, H, F, o, idx, cnt);
        break;
    case 2:
        hipLaunchKernelGGL((k_pass2<2>), dim3(blocks_for(2 * n)), dim3(BLOCK), 0,
                           c->stream, v, P, E, H, F, o, idx, cnt);
        break;
    default:
        hipLaunchKernelGGL((k_pass2<1>), dim3(blocks_for(n)), dim3(BLOCK), 0,
                           c->stream, v, P, E, H, F, o, idx, cnt);
    }
}

// Size-class dispatch applies to the float64 quadratic fits.
bool classes_on(const lp_ctx* c)
{
    return c->classes && c->cfg.fit_order == 2 && c->cfg.precision == LP_FP64;
}

// Pass 1 of a step: the size classes with their lanes, or one launch.
void run_pass1(lp_ctx* c, const View& v, const StepOut& so, int fq)
{
    if (classes_on(c)) {
        classify(c, v);
        for (int k = 0; k < NCLASS; ++k) launch_pass1_class(c, k, c->cls_lpp1[k], v, so, fq);
    } else {
        launch_pass1(c, c->lpp1, v, so, fq);
    }
}

void run_pass2(lp_ctx* c, const View& v, const RhsOut& o)
{
    if (classes_on(c)) {
        for (int k = 0; k < NCLASS; ++k) launch_pass2_class(c, k, c->cls_lpp2[k], v, o);
    } else {
        launch_pass2(c, c->lpp2, v, o);
    }
}

}  // namespace

lp_status fit_generic(lp_ctx* c, const double* const st[7], const double* f,
                      int k, const int32_t* msign, const int32_t* gzero,
                      double* coef, uint8_t* flags)
{
    lp_status r = need_stencils(c);
    if (r != LP_OK) return r;
    Work& w = c->w;
    const int64_t n = c->n;
    View v = make_view(c, st);
    GenericFields F;
    F.f = f;
    F.k = k;
    for (int q = 0; q < 8; ++q) {
        F.msign[q] = q < k ? msign[q] : 0;
        F.gzero[q] = q < k ? gzero[q] : 0;
    }
    uint8_t* fl = flags ? flags : w.flags;
    const int fq = (c->cfg.debug_flags & LP_DEBUG_QR_FIT) ? 1 : 0;
    redo_reset(c);
    if (n > 0 && c->cfg.fit_order == 3) {
        launch_fit3_generic(c, v, F, coef, fl);
    } else if (n > 0) {
        const dim3 gb(blocks_for(n)), bb(BLOCK);
#define LP_FIT_CASE(K)                                                          \
    case K:                                                                     \
        hipLaunchKernelGGL(k_fit_generic<K>, gb, bb, 0, c->stream, v, F, coef, \
                           fl, w.redo, w.redo_n, fq);                           \
        break;
        switch (k) {
            LP_FIT_CASE(1) LP_FIT_CASE(2) LP_FIT_CASE(3) LP_FIT_CASE(4)
            LP_FIT_CASE(5) LP_FIT_CASE(6) LP_FIT_CASE(7) LP_FIT_CASE(8)
        default: break;
        }
#undef LP_FIT_CASE
        hipLaunchKernelGGL(k_fit_generic_qr, dim3(QR_BLOCKS), dim3(QR_TPB), 0,
                           c->stream, v, F, coef, fl, w.redo, w.redo_n,
                           w.cnt);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "fit launch");
    return LP_OK;
}

static RhsOut rhs_out(lp_ctx* c, double* acc, double* dVdt, double* grad)
{
    RhsOut o;
    o.acc = acc;
    o.dVdt = dVdt;
    o.grad = grad;
    o.flags = c->w.flags;
    for (int a = 0; a < 7; ++a) o.out[a] = nullptr;
    o.dt = 0.0;
    o.err = c->w.err;
    o.cnt = c->w.cnt;
    o.reflect = c->cfg.wall_reflect;
    return o;
}

lp_status rhs_from_coef(lp_ctx* c, const double* const st[7],
                        const double* coef_u, double* dVdt, double* acc,
                        double* diag, double* grad, uint8_t* flags)
{
    lp_status r = need_stencils(c);
    if (r != LP_OK) return r;
    Work& w = c->w;
    const int64_t n = c->n;
    View v = make_view(c, st);
    StepOut so{w.P, w.eta, w.hand, w.flags, diag, nullptr};
    const int fq = (c->cfg.debug_flags & LP_DEBUG_QR_FIT) ? 1 : 0;
    redo_reset(c);
    if (n > 0) {
        hipLaunchKernelGGL(k_closure_coef, dim3(blocks_for(n)), dim3(BLOCK), 0,
                           c->stream, v, coef_u, so, w.redo, w.redo_n, fq);
        RhsOut o = rhs_out(c, acc, dVdt, grad);
        if (c->cfg.fit_order == 3) {
            launch_pass2_cubic(c, v, w.P, w.eta, w.hand, o);
        } else {
            launch_pass2(c, c->lpp2, v, o);
            hipLaunchKernelGGL(k_pass2_qr, dim3(QR_BLOCKS), dim3(QR_TPB), 0,
                               c->stream, v, (const double*)w.P, (const double*)w.eta,
                               (const double*)w.hand, (const int32_t*)w.redo,
                               (const unsigned int*)w.redo_n, o);
        }
        if (flags)
            hipLaunchKernelGGL(k_copy_u8, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, n, w.flags, flags);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "rhs launch");
    return LP_OK;
}

lp_status step_rhs(lp_ctx* c, const double* const st[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    View v = make_view(c, st);
    StepOut so{w.P, w.eta, w.hand, w.flags, nullptr, nullptr};
    const int fq = (c->cfg.debug_flags & LP_DEBUG_QR_FIT) ? 1 : 0;
    redo_reset(c);
    if (n > 0) {
        prof_mark(c, 3, false);
        if (c->cfg.fit_order == 3)
            launch_pass1_cubic(c, v, so);
        else if (c->cfg.precision == LP_FP32_REFINED && !fq) {
            const int mo = c->map_ok ? 1 : 0;
            if (c->cfg.weight == LP_W_UNIT)
                hipLaunchKernelGGL(k_pass1_ref<true>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                                   c->stream, v, so, w.uf, w.redo, w.redo_n, mo);
            else
                hipLaunchKernelGGL(k_pass1_ref<false>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                                   c->stream, v, so, w.uf, w.redo, w.redo_n, mo);
        }
        else
            run_pass1(c, v, so, fq);
        prof_mark(c, 3, true);
        prof_mark(c, 4, false);
        hipLaunchKernelGGL(k_pass1_qr, dim3(QR_BLOCKS), dim3(QR_TPB), 0,
                           c->stream, v, so, (const int32_t*)w.redo,
                           (const unsigned int*)w.redo_n, w.cnt);
        prof_mark(c, 4, true);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "pass-1 launch");
    return LP_OK;
}

lp_status step_pass1_coef(lp_ctx* c, const double* const st[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    View v = make_view(c, st);
    StepOut so{w.P, w.eta, w.hand, w.flags, nullptr, w.coefu};
    redo_reset(c);
    if (n > 0) {
        // the pass-2 fit of these stencils may run by size class
        if (classes_on(c)) classify(c, v);
        launch_pass1(c, c->lpp1, v, so, 0);
        hipLaunchKernelGGL(k_pass1_qr, dim3(QR_BLOCKS), dim3(QR_TPB), 0,
                           c->stream, v, so, (const int32_t*)w.redo,
                           (const unsigned int*)w.redo_n, w.cnt);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "adjoint pass-1 launch");
    return LP_OK;
}

lp_status step_pass2(lp_ctx* c, const double* const st[7], double dt,
                     double* const out[7], double* acc, double* dVdt, bool fp64)
{
    Work& w = c->w;
    const int64_t n = c->n;
    View v = make_view(c, st);
    RhsOut o = rhs_out(c, acc, dVdt, nullptr);
    for (int a = 0; a < 7; ++a) o.out[a] = out ? out[a] : nullptr;
    o.dt = dt;
    if (n > 0) {
        prof_mark(c, 5, false);
        if (c->cfg.fit_order == 3)
            launch_pass2_cubic(c, v, w.P, w.eta, w.hand, o);
        else if (c->cfg.precision == LP_FP32_REFINED && !fp64) {
            const int mo = c->map_ok ? 1 : 0;
            if (c->cfg.weight == LP_W_UNIT)
                hipLaunchKernelGGL(k_pass2_ref<true>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                                   c->stream, v, (const double*)w.P, (const double*)w.eta,
                                   (const double*)w.hand, (const float*)w.uf,
                                   (const uint8_t*)w.flags, o, mo);
            else
                hipLaunchKernelGGL(k_pass2_ref<false>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                                   c->stream, v, (const double*)w.P, (const double*)w.eta,
                                   (const double*)w.hand, (const float*)w.uf,
                                   (const uint8_t*)w.flags, o, mo);
        }
        else
            run_pass2(c, v, o);
        prof_mark(c, 5, true);
        prof_mark(c, 6, false);
        hipLaunchKernelGGL(k_pass2_qr, dim3(QR_BLOCKS), dim3(QR_TPB), 0,
                           c->stream, v, (const double*)w.P, (const double*)w.eta,
                           (const double*)w.hand, (const int32_t*)w.redo,
                           (const unsigned int*)w.redo_n, o);
        prof_mark(c, 6, true);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "pass-2 launch");
    return LP_OK;
}

lp_status step_update(lp_ctx* c, const double* const st[7], double dt,
                      double* const out[7])
{
    return step_pass2(c, st, dt, out, c->w.acc, c->w.dVdt);
}

lp_status autotune_fits(lp_ctx* c, const double* const st[7], int32_t* choice)
{
    if (c->cfg.fit_order == 3) {   // a wavefront per particle: nothing to tune
        if (choice) choice[0] = choice[1] = 1;
        return LP_OK;
    }
    Work& w = c->w;
    View v = make_view(c, st);
    StepOut so{w.P, w.eta, w.hand, w.flags, nullptr, nullptr};
    RhsOut o = rhs_out(c, w.acc, w.dVdt, nullptr);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    // best of three timings of one launch sequence
    auto timed = [&](auto&& launch) -> float {
        float t = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            redo_reset(c);
            e = hipEventRecord(e0, c->stream);
            launch();
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            t = ms < t ? ms : t;
        }
        return t;
    };
    const int cand[3] = {1, 2, 4};
    // one launch over all particles, 1 (LDS-staged when the tile map is
    // current), 2 or 4 lanes per particle
    float best1 = 1e30f, best2 = 1e30f;
    int pick1 = 1, pick2 = 1;
    for (int q = 0; q < 3 && e == hipSuccess; ++q) {
        const float t = timed([&] { launch_pass1(c, cand[q], v, so, 0); });
        if (t < best1) { best1 = t; pick1 = cand[q]; }
    }
    // pass 2 needs the pass-1 outputs
    if (e == hipSuccess) {
        redo_reset(c);
        launch_pass1(c, pick1, v, so, 0);
    }
    for (int q = 0; q < 3 && e == hipSuccess; ++q) {
        const float t = timed([&] { launch_pass2(c, cand[q], v, o); });
        if (t < best2) { best2 = t; pick2 = cand[q]; }
    }
    // by stencil size class (float64 quadratic fits): each class with its
    // own lanes per particle
    bool use_classes = false;
    float cb1[NCLASS] = {0.f, 0.f, 0.f}, cb2[NCLASS] = {0.f, 0.f, 0.f};
    int cp1[NCLASS] = {1, 1, 1}, cp2[NCLASS] = {1, 1, 1};
    uint32_t counts[4] = {0, 0, 0, 0};
    if (e == hipSuccess && c->cfg.precision == LP_FP64 && c->n > 0) {
        classify(c, v);
        e = hipMemcpyAsync(counts, w.cls_cnt, sizeof(uint32_t) * NCLASS,
                           hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        for (int k = 0; k < NCLASS && e == hipSuccess; ++k) {
            cb1[k] = 1e30f;
            if (counts[k] == 0) {
                cb1[k] = 0.f;
                continue;
            }
            for (int q = (k == NCLASS - 1 ? -1 : 0); q < 3 && e == hipSuccess; ++q) {
                const int l = q < 0 ? 0 : cand[q];   // 0: staged tile kernel
                const float t = timed([&] { launch_pass1_class(c, k, l, v, so, 0); });
                if (t < cb1[k]) { cb1[k] = t; cp1[k] = l; }
            }
        }
        if (e == hipSuccess) {
            redo_reset(c);
            launch_pass1(c, pick1, v, so, 0);
        }
        for (int k = 0; k < NCLASS && e == hipSuccess; ++k) {
            cb2[k] = 1e30f;
            if (counts[k] == 0) {
                cb2[k] = 0.f;
                continue;
            }
            for (int q = (k == NCLASS - 1 ? -1 : 0); q < 3 && e == hipSuccess; ++q) {
                const int l = q < 0 ? 0 : cand[q];
                const float t = timed([&] { launch_pass2_class(c, k, l, v, o); });
                if (t < cb2[k]) { cb2[k] = t; cp2[k] = l; }
            }
        }
        float tot = 0.f;
        for (int k = 0; k < NCLASS; ++k) tot += cb1[k] + cb2[k];
        use_classes = tot < best1 + best2;
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(c, e, "autotune");
    c->lpp1 = pick1;
    c->lpp2 = pick2;
    c->classes = use_classes;
    c->tune_ms[0] = best1;
    c->tune_ms[1] = best2;
    for (int k = 0; k < NCLASS; ++k) {
        c->cls_lpp1[k] = cp1[k];
        c->cls_lpp2[k] = cp2[k];
        c->cls_count[k] = counts[k];
        c->tune_ms[2 + k] = cb1[k];
        c->tune_ms[5 + k] = cb2[k];
    }
    if (choice) {
        choice[0] = pick1;
        choice[1] = pick2;
    }
    return LP_OK;
}

}  // namespace lp
