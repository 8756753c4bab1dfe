// Cubic (third-order, 19-unknown) least-squares fits: the higher-order
// fits the paper lists as further work, for the fits of Sec. 3.1 step 7.
// The Taylor row gains the cubic monomials divided by the factorials of
// their exponents (each coefficient is the matching third derivative times
// h^3); the step uses the first and second derivatives as before.
//
// One wavefront per particle: lane t holds fit row t (the stencil rows in
// the order of the stencil walk, then the ghost rows), so a stencil of up
// to 64 rows is one register column per unknown.  Householder QR runs
// across the lanes (each reflector: one wave-wide sum per remaining
// column and right-hand side), the back substitution broadcasts one
// coefficient per step.  Stencils with fewer than 19 rows, or whose
// min |r_jj| / max |r_jj| is below the fallback tolerance, are refitted
// with the 9 quadratic columns (FLAG_QUAD), then with the 3 linear ones
// (FLAG_LINEAR), as the quadratic fit does.
#include "lp_finish.h"

namespace lp {

namespace {

constexpr int NC3 = 19;
constexpr int WAVES = BLOCK / 64;

inline unsigned int blocks_for_waves(int64_t n)
{
    return (unsigned int)((n + WAVES - 1) / WAVES);
}

// one DPP lane permutation of a double (both halves), within rows of 16
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x)
{
    const int lo = __double2loint(x), hi = __double2hiint(x);
    const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
    const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double readlane_f64(double x, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, the same value in every lane.  Within each row
// of 16 lanes: neighbour and pair swaps inside quads, then the half-row
// and row mirrors (each stage adds the same two operands in both partner
// lanes); the four row sums are then read as scalars and added in one
// fixed order.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_f64<0xB1>(x);    // quad_perm [1, 0, 3, 2]
    x += dpp_f64<0x4E>(x);    // quad_perm [2, 3, 0, 1]
    x += dpp_f64<0x141>(x);   // row_half_mirror
    x += dpp_f64<0x140>(x);   // row_mirror
    return (readlane_f64(x, 0) + readlane_f64(x, 16)) +
           (readlane_f64(x, 32) + readlane_f64(x, 48));
}

// list index of the k-th set bit (0-based) of the keep mask, -1 if none
__device__ __forceinline__ int mask_select(const Rec& r, int k)
{
#pragma unroll
    for (int w = 0; w < MASK_WORDS; ++w) {
        const int c = __popcll(r.mask[w]);
        if (k < c) {
            uint64_t b = r.mask[w];
            for (int s = 0; s < k; ++s) b &= b - 1;
            return 64 * w + __builtin_ctzll(b);
        }
        k -= c;
    }
    return -1;
}

__device__ __forceinline__ void taylor_row3(double ex, double ey, double ez,
                                            double (&a)[NC3])
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
    a[9] = ex * ex * ex / 6.0;
    a[10] = ey * ey * ey / 6.0;
    a[11] = ez * ez * ez / 6.0;
    a[12] = 0.5 * ex * ex * ey;
    a[13] = 0.5 * ex * ex * ez;
    a[14] = 0.5 * ey * ey * ex;
    a[15] = 0.5 * ey * ey * ez;
    a[16] = 0.5 * ez * ez * ex;
    a[17] = 0.5 * ez * ez * ey;
    a[18] = ex * ey * ez;
}

// Row `lane` of particle i's fit: the weighted Taylor row and the point
// (nullptr for a ghost row; rows beyond the last are zero).  Returns the
// square root of the weight (0 for an empty row).
__device__ __forceinline__ double lane_row(const View& v, const GridInfo& g, int64_t i,
                                           const Rec& r, int lane, double (&a)[NC3],
                                           Pt& pt, bool& ghost)
{
    const int64_t n = v.n;
    const double xi = v.x[i], yi = v.y[i], zi = v.z[i];
    ghost = false;
    const int ng = __popc((unsigned)r.gm & 0xFFu);
    if (lane < r.m) {
        if (r.mode & MODE_SORTED) {
            pt = id_point(v, g, v.hsten[(int64_t)lane * n + i], xi, yi);
        } else {
            const int k = mask_select(r, lane);
            pt = list_point(v, g, v.vl[(int64_t)k * n + i], xi, yi);
        }
        const double dx = dsub(pt.x, xi), dy = dsub(pt.y, yi), dz = dsub(pt.z, zi);
        taylor_row3(dx * g.inv_h, dy * g.inv_h, dz * g.inv_h, a);
        double sw = 1.0;
        if (v.weight == LP_W_GAUSS) sw = sqrt(exp(-4.0 * (dx * dx + dy * dy + dz * dz) / g.R2));
#pragma unroll
        for (int q = 0; q < NC3; ++q) a[q] *= sw;
        return sw;
    }
    if (lane < r.m + ng) {
        // ghost rows in ascending octant order
        unsigned gm = (unsigned)r.gm & 0xFFu;
        for (int s = 0; s < lane - r.m; ++s) gm &= gm - 1;
        const int o = __builtin_ctz(gm);
        double sx, sy, sz;
        ghost_offset(o, sx, sy, sz);
        taylor_row3(sx, sy, sz, a);
        double sw = 1.0;
        if (v.weight == LP_W_GAUSS) sw = sqrt(exp(-12.0 * g.h * g.h / g.R2));
#pragma unroll
        for (int q = 0; q < NC3; ++q) a[q] *= sw;
        ghost = true;
        return sw;
    }
#pragma unroll
    for (int q = 0; q < NC3; ++q) a[q] = 0.0;
    return 0.0;
}

// Householder QR of the first NC columns of the lane-distributed rows
// (rows 0..m-1 in lanes 0..m-1) applied to NF right-hand sides; R and
// Q^T b stay in place (row j of R in lane j).  rd: diagonal of R (the
// same in every lane).  Returns min |r_jj| / max |r_jj| (0 when a column
// vanishes).
template <int NC, int NF>
__device__ __forceinline__ double wave_house(int lane, int m, double (&a)[NC3],
                                             double (&b)[NF], double (&rd)[NC3])
{
    double rmin = INFINITY, rmax = 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
        const bool act = lane >= j && lane < m;
        const double s = wave_sum(act ? a[j] * a[j] : 0.0);
        const double nrm = sqrt(s);
        const double ajj = __shfl(a[j], j);
        if (nrm == 0.0) {
            rd[j] = 0.0;
            rmin = 0.0;
            continue;
        }
        const double alpha = ajj >= 0.0 ? -nrm : nrm;
        if (lane == j) a[j] = ajj - alpha;
        const double vtv = 2.0 * nrm * (nrm + fabs(ajj));
        const double vj = act ? a[j] : 0.0;
#pragma unroll
        for (int l = j + 1; l < NC; ++l) {
            const double f = 2.0 * wave_sum(vj * a[l]) / vtv;
            if (act) a[l] -= f * vj;
        }
#pragma unroll
        for (int l = 0; l < NF; ++l) {
            const double f = 2.0 * wave_sum(vj * b[l]) / vtv;
            if (act) b[l] -= f * vj;
        }
        rd[j] = alpha;
        const double ar = fabs(alpha);
        rmin = fmin(rmin, ar);
        rmax = fmax(rmax, ar);
    }
    return rmax > 0.0 ? rmin / rmax : 0.0;
}

// R x = Q^T b for right-hand side `f` after wave_house; x (per unit h) is
// the same in every lane.
template <int NC, int NF>
__device__ __forceinline__ void wave_backsolve(int lane, const double (&a)[NC3],
                                               const double (&b)[NF], int f,
                                               const double (&rd)[NC3], double (&x)[NC3])
{
#pragma unroll
    for (int q = 0; q < NC3; ++q) x[q] = 0.0;
#pragma unroll
    for (int c = NC - 1; c >= 0; --c) {
        double acc = b[f];
#pragma unroll
        for (int q = c + 1; q < NC; ++q) acc -= a[q] * x[q];
        const double xc = __shfl(acc, c);
        x[c] = rd[c] != 0.0 ? xc / rd[c] : 0.0;
    }
}

// The fit of NF fields at particle i with the 19 -> 9 -> 3 column
// fallback.  vals(pt, ghost, out): the NF field values of the row's point
// minus the particle's own (ghost rows: the ghost values minus the own).
// coef[f][q]: derivative q (first 9) of field f, scaled by 1/h, 1/h^2.
template <int NF, class Vals>
__device__ __forceinline__ uint8_t wave_fit3(const View& v, const GridInfo& g,
                                             int64_t i, const Rec& r, int lane,
                                             Vals&& vals, double (&coef)[NF][9])
{
    const int m = r.m + __popc((unsigned)r.gm & 0xFFu);
    double a[NC3], b[NF], rd[NC3], x[NC3];
    auto load = [&]() {
        Pt pt;
        bool ghost;
        const double sw = lane_row(v, g, i, r, lane, a, pt, ghost);
        double d[NF];
        if (lane < m) vals(ghost ? nullptr : &pt, d);
#pragma unroll
        for (int f = 0; f < NF; ++f) b[f] = lane < m ? sw * d[f] : 0.0;
    };
    uint8_t fl = 0;
    int nc = 0;
    if (m >= NC3) {
        load();
        if (wave_house<NC3, NF>(lane, m, a, b, rd) >= v.fallback_tol) nc = NC3;
    }
    if (nc == 0) {
        fl |= FLAG_QUAD;
        if (m >= 9) {
            load();
            if (wave_house<9, NF>(lane, m, a, b, rd) >= v.fallback_tol) nc = 9;
        }
    }
    if (nc == 0) {
        fl |= FLAG_LINEAR;
        if (m >= 3) {
            load();
            wave_house<3, NF>(lane, m, a, b, rd);
            nc = 3;
        }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (nc == NC3) wave_backsolve<NC3, NF>(lane, a, b, f, rd, x);
        else if (nc == 9) wave_backsolve<9, NF>(lane, a, b, f, rd, x);
        else if (nc == 3) wave_backsolve<3, NF>(lane, a, b, f, rd, x);
        else
#pragma unroll
            for (int q = 0; q < NC3; ++q) x[q] = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) coef[f][q] = x[q] * (q < 3 ? g.inv_h : g.inv_h * g.inv_h);
    }
    return fl;
}

// ---- lp_fit_derivs -------------------------------------------------------

template <int NF>
__global__ __launch_bounds__(BLOCK) void k_fit3_generic(View v, GenericFields F,
                                                        double* coef, uint8_t* flags)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * WAVES + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (i >= v.n) return;
    const int64_t n = v.n;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    const Rec r = load_rec(v, i);
    double own[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) own[f] = F.f[(int64_t)f * n + i];
    auto vals = [&](const Pt* p, double (&d)[NF]) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            double fj;
            if (!p) fj = F.gzero[f] ? 0.0 : own[f];
            else if (p->mirror) fj = (double)F.msign[f] * F.f[(int64_t)f * n + p->src];
            else fj = F.f[(int64_t)f * n + p->src];
            d[f] = fj - own[f];
        }
    };
    double c[NF][9];
    const uint8_t fl = wave_fit3<NF>(v, g, i, r, lane, vals, c);
    if (lane != 0) return;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 9; ++q) coef[((int64_t)f * 9 + q) * n + i] = c[f][q];
    if (flags) flags[i] = fl;
}

// ---- pass 1: fit of u, v, w and the closure ------------------------------

__global__ __launch_bounds__(BLOCK) void k_pass1_cubic(View v, StepOut o)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * WAVES + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (i >= v.n) return;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const Rec r = load_rec(v, i);
    const double ui = v.u[i], vi = v.v[i], wi = v.w[i];
    auto vals = [&](const Pt* p, double (&d)[3]) {
        if (!p) {   // ghosts carry the particle's velocity
            d[0] = d[1] = d[2] = 0.0;
            return;
        }
        double uj, vj, wj;
        point_velocity(v, *p, uj, vj, wj);
        d[0] = uj - ui;
        d[1] = vj - vi;
        d[2] = wj - wi;
    };
    double c3[3][9];
    const uint8_t fl = wave_fit3<3>(v, g, i, r, lane, vals, c3);
    if (lane != 0) return;
    double c[27], ginv3[27];
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int q = 0; q < 9; ++q) c[f * 9 + q] = c3[f][q];
#pragma unroll
    for (int q = 0; q < 27; ++q) ginv3[q] = 0.0;
    finish_pass1(v, v.prm[s], i, c, ginv3, false, fl, o);
}

// ---- pass 2: fit of P and eta, right-hand side, update ---------------------

__global__ __launch_bounds__(BLOCK) void k_pass2_cubic(View v, const double* P,
                                                       const double* eta,
                                                       const double* hand, RhsOut o)
{
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * WAVES + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (i >= v.n) return;
    const int64_t n = v.n;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const lp_params& prm = v.prm[s];
    const Rec r = load_rec(v, i);
    const double Pi = P[i], Ei = eta[i];
    auto vals = [&](const Pt* p, double (&d)[2]) {
        double Pj, Ej;
        pass2_values(v, P, eta, p, prm, Pj, Ej);
        d[0] = Pj - Pi;
        d[1] = Ej - Ei;
    };
    double c2[2][9];
    const uint8_t fl = wave_fit3<2>(v, g, i, r, lane, vals, c2);
    if (lane != 0) return;
    // the fit's fallback bits next to the regime of the closure
    o.flags[i] = (uint8_t)((o.flags[i] & 6) | fl);
    const double gP[3] = {c2[0][0], c2[0][1], c2[0][2]};
    const double gE[3] = {c2[1][0], c2[1][1], c2[1][2]};
    double hv[11];
    load_hand_tail(hand, n, i, Ei, hv);
    finish_rhs(v, prm, i, hv, gP, gE, o);
}

}  // namespace

void launch_fit3_generic(lp_ctx* c, const View& v, const GenericFields& F, double* coef,
                         uint8_t* flags)
{
    const dim3 gb(blocks_for_waves(c->n)), bb(BLOCK);
#define LP_FIT3_CASE(K)                                                              \
    case K:                                                                          \
        hipLaunchKernelGGL(k_fit3_generic<K>, gb, bb, 0, c->stream, v, F, coef, flags); \
        break;
    switch (F.k) {
        LP_FIT3_CASE(1) LP_FIT3_CASE(2) LP_FIT3_CASE(3) LP_FIT3_CASE(4)
        LP_FIT3_CASE(5) LP_FIT3_CASE(6) LP_FIT3_CASE(7) LP_FIT3_CASE(8)
    default: break;
    }
#undef LP_FIT3_CASE
}

void launch_pass1_cubic(lp_ctx* c, const View& v, const StepOut& o)
{
    hipLaunchKernelGGL(k_pass1_cubic, dim3(blocks_for_waves(c->n)), dim3(BLOCK), 0,
                       c->stream, v, o);
}

void launch_pass2_cubic(lp_ctx* c, const View& v, const double* P, const double* eta,
                        const double* hand, const RhsOut& o)
{
    hipLaunchKernelGGL(k_pass2_cubic, dim3(blocks_for_waves(c->n)), dim3(BLOCK), 0,
                       c->stream, v, P, eta, hand, o);
}

}  // namespace lp
