// Cubic (third-order, 19-unknown) least-squares fits: the higher-order
// fits the paper lists as further work, for the fits of Sec. 3.1 step 7.
// The Taylor row gains the cubic monomials divided by the factorials of
// their exponents (each coefficient is the matching third derivative times
// h^3); the step uses the first and second derivatives as before.
//
// Sixteen lanes per particle (one DPP row; four particles per wavefront):
// lane s of a particle's group holds fit rows s, s + 16, s + 32 and s + 48
// (the stencil rows in the order of the stencil walk, then the ghost
// rows), so a stencil of up to 64 rows is four register columns per
// unknown.  Householder QR runs across the group: each reflector sums over
// the lane's four rows, then over the sixteen lanes with DPP steps inside
// the row; the pivot and, in the back substitution, each coefficient are
// broadcast from the lane that holds their row.  Stencils with fewer than
// 19 rows, or whose min |r_jj| / max |r_jj| is below the fallback
// tolerance, are refitted with the 9 quadratic columns (FLAG_QUAD), then
// with the 3 linear ones (FLAG_LINEAR), as the quadratic fit does.
#include <type_traits>

#include "lp_finish.h"

namespace lp {

namespace {

constexpr int NC3 = 19;
constexpr int GROUP = 16;             // lanes per particle
constexpr int SLOTS = 4;              // rows per lane: up to 64 rows
constexpr int PPB = BLOCK / GROUP;    // particles per block

inline unsigned int blocks_for_groups(int64_t n)
{
    return (unsigned int)((n + PPB - 1) / PPB);
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

// Sum over the 16 lanes of a group, the same value in every lane: swaps
// of neighbours and pairs inside quads, then the half-row and row mirrors
// (each stage adds the same two operands in both partner lanes).
__device__ __forceinline__ double group_sum(double x)
{
    x += dpp_f64<0xB1>(x);    // quad_perm [1, 0, 3, 2]
    x += dpp_f64<0x4E>(x);    // quad_perm [2, 3, 0, 1]
    x += dpp_f64<0x141>(x);   // row_half_mirror
    x += dpp_f64<0x140>(x);   // row_mirror
    return x;
}

// f(integral_constant<int, K>) for K = B .. E-1, in order
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// lane SRC's value in every lane of the group (row broadcast)
template <int SRC>
__device__ __forceinline__ double group_bcast(double x)
{
    return dpp_f64<0x150 + SRC>(x);
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

// Fit row `row` of particle i: the weighted Taylor row and its point
// (ghost rows: ghost = true; rows beyond the last are zero).  Returns the
// square root of the weight (0 for an empty row).
__device__ __forceinline__ double fit_row(const View& v, const GridInfo& g, int64_t i,
                                          const Rec& r, int row, double (&a)[NC3], Pt& pt,
                                          bool& ghost)
{
    const int64_t n = v.n;
    const double xi = v.x[i], yi = v.y[i], zi = v.z[i];
    ghost = false;
    const int ng = __popc((unsigned)r.gm & 0xFFu);
    if (row < r.m) {
        if (r.mode & MODE_SORTED) {
            pt = id_point(v, g, v.hsten[(int64_t)row * n + i], xi, yi);
        } else {
            const int k = mask_select(r, row);
            pt = list_point(v, g, v.vl[vl_at(n, i, k)], xi, yi);
        }
        const double dx = dsub(pt.x, xi), dy = dsub(pt.y, yi), dz = dsub(pt.z, zi);
        taylor_row3(dx * g.inv_h, dy * g.inv_h, dz * g.inv_h, a);
        double sw = 1.0;
        if (v.weight == LP_W_GAUSS) sw = sqrt(exp(-4.0 * (dx * dx + dy * dy + dz * dz) / g.R2));
#pragma unroll
        for (int q = 0; q < NC3; ++q) a[q] *= sw;
        return sw;
    }
    if (row < r.m + ng) {
        // ghost rows in ascending octant order
        unsigned gm = (unsigned)r.gm & 0xFFu;
        for (int s = 0; s < row - r.m; ++s) gm &= gm - 1;
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

// Householder QR of the first NC columns of the group's rows (row
// 16 q + s in slot q of lane s) applied to NF right-hand sides; R and
// Q^T b stay in place, r_jj in rdiag of the lane holding row j.  Returns
// min |r_jj| / max |r_jj| (0 when a column vanishes), the same in every
// lane of the group.
template <int NC, int NF>
__device__ __forceinline__ double group_house(int sl, int m, double (&a)[SLOTS][NC3],
                                              double (&b)[SLOTS][NF],
                                              double (&rdiag)[SLOTS])
{
    double rmin = INFINITY, rmax = 0.0;
    static_for<0, NC>([&](auto J) {
        constexpr int j = decltype(J)::value;
        bool act[SLOTS];
        double part = 0.0;
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            const int row = GROUP * q + sl;
            act[q] = row >= j && row < m;
            part += act[q] ? a[q][j] * a[q][j] : 0.0;
        }
        const double nrm = sqrt(group_sum(part));
        const double ajj = group_bcast<j % GROUP>(a[j / GROUP][j]);
        if (nrm == 0.0) {
            if (sl == j % GROUP) rdiag[j / GROUP] = 0.0;
            rmin = 0.0;
            return;
        }
        const double alpha = ajj >= 0.0 ? -nrm : nrm;
        if (sl == j % GROUP) a[j / GROUP][j] = ajj - alpha;
        const double vtv = 2.0 * nrm * (nrm + fabs(ajj));
        const double s2 = 2.0 / vtv;   // one division per column step
        double vj[SLOTS];
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) vj[q] = act[q] ? a[q][j] : 0.0;
#pragma unroll
        for (int l = j + 1; l < NC; ++l) {
            double d = 0.0;
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) d += vj[q] * a[q][l];
            const double f = group_sum(d) * s2;
            // vj is 0 on the inactive rows, which the update leaves as
            // they are
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) a[q][l] -= f * vj[q];
        }
#pragma unroll
        for (int l = 0; l < NF; ++l) {
            double d = 0.0;
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) d += vj[q] * b[q][l];
            const double f = group_sum(d) * s2;
#pragma unroll
            for (int q = 0; q < SLOTS; ++q) b[q][l] -= f * vj[q];
        }
        if (sl == j % GROUP) rdiag[j / GROUP] = alpha;
        const double ar = fabs(alpha);
        rmin = fmin(rmin, ar);
        rmax = fmax(rmax, ar);
    });
    return rmax > 0.0 ? rmin / rmax : 0.0;
}

// R x = Q^T b for right-hand side `f` after group_house; x (per unit h) is
// the same in every lane of the group.
template <int NC, int NF>
__device__ __forceinline__ void group_backsolve(const double (&a)[SLOTS][NC3],
                                                const double (&b)[SLOTS][NF], int f,
                                                const double (&rdiag)[SLOTS],
                                                double (&x)[NC3])
{
#pragma unroll
    for (int q = 0; q < NC3; ++q) x[q] = 0.0;
    double rinv[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) rinv[q] = rdiag[q] != 0.0 ? 1.0 / rdiag[q] : 0.0;
    static_for<0, NC>([&](auto K) {
        constexpr int c = NC - 1 - decltype(K)::value;
        // computed in every lane; the lane holding row c has the right one
        double acc = b[c / GROUP][f];
#pragma unroll
        for (int q = c + 1; q < NC; ++q) acc -= a[c / GROUP][q] * x[q];
        x[c] = group_bcast<c % GROUP>(acc * rinv[c / GROUP]);
    });
}

// The fit of NF fields at particle i with the 19 -> 9 -> 3 column
// fallback.  vals(pt or nullptr for a ghost, out): the NF field values of
// the row's point minus the particle's own.  coef[f][q]: derivative q
// (first 9) of field f, scaled by 1/h, 1/h^2.
template <int NF, class Vals>
__device__ __forceinline__ uint8_t group_fit3(const View& v, const GridInfo& g,
                                              int64_t i, const Rec& r, int sl,
                                              Vals&& vals, double (&coef)[NF][9])
{
    const int m = r.m + __popc((unsigned)r.gm & 0xFFu);
    double a[SLOTS][NC3], b[SLOTS][NF], rdiag[SLOTS], x[NC3];
    auto load = [&]() {
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            const int row = GROUP * q + sl;
            Pt pt;
            bool ghost;
            const double sw = fit_row(v, g, i, r, row, a[q], pt, ghost);
            double d[NF];
            if (row < m) vals(ghost ? nullptr : &pt, d);
#pragma unroll
            for (int f = 0; f < NF; ++f) b[q][f] = row < m ? sw * d[f] : 0.0;
            rdiag[q] = 0.0;
        }
    };
    uint8_t fl = 0;
    int nc = 0;
    const bool enough_real = r.m >= v.min_real;   // else the linear fit
    if (m >= NC3 && enough_real) {
        load();
        if (group_house<NC3, NF>(sl, m, a, b, rdiag) >= v.fallback_tol) nc = NC3;
    }
    if (nc == 0) {
        fl |= FLAG_QUAD;
        if (m >= 9 && enough_real) {
            load();
            if (group_house<9, NF>(sl, m, a, b, rdiag) >= v.fallback_tol) nc = 9;
        }
    }
    if (nc == 0) {
        fl |= FLAG_LINEAR;
        if (m >= 3) {
            load();
            group_house<3, NF>(sl, m, a, b, rdiag);
            nc = 3;
        }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (nc == NC3) group_backsolve<NC3, NF>(a, b, f, rdiag, x);
        else if (nc == 9) group_backsolve<9, NF>(a, b, f, rdiag, x);
        else if (nc == 3) group_backsolve<3, NF>(a, b, f, rdiag, x);
        else
#pragma unroll
            for (int q = 0; q < NC3; ++q) x[q] = 0.0;
#pragma unroll
        for (int q = 0; q < 9; ++q) coef[f][q] = x[q] * (q < 3 ? g.inv_h : g.inv_h * g.inv_h);
    }
    return fl;
}

__device__ __forceinline__ int64_t group_particle(int& sl)
{
    sl = threadIdx.x % GROUP;
    return xcd_block(blockIdx.x, gridDim.x) * PPB + threadIdx.x / GROUP;
}

// ---- lp_fit_derivs -------------------------------------------------------

template <int NF>
__global__ __launch_bounds__(BLOCK) void k_fit3_generic(View v, GenericFields F,
                                                        double* coef, uint8_t* flags)
{
    int sl;
    const int64_t i = group_particle(sl);
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
    const uint8_t fl = group_fit3<NF>(v, g, i, r, sl, vals, c);
    if (sl != 0) return;
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int q = 0; q < 9; ++q) coef[((int64_t)f * 9 + q) * n + i] = c[f][q];
    if (flags) flags[i] = fl;
}

// ---- pass 1: fit of u, v, w and the closure ------------------------------

__global__ __launch_bounds__(BLOCK) void k_pass1_cubic(View v, StepOut o)
{
    int sl;
    const int64_t i = group_particle(sl);
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
    const uint8_t fl = group_fit3<3>(v, g, i, r, sl, vals, c3);
    if (sl != 0) return;
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
    int sl;
    const int64_t i = group_particle(sl);
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
    const uint8_t fl = group_fit3<2>(v, g, i, r, sl, vals, c2);
    if (sl != 0) return;
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
    const dim3 gb(blocks_for_groups(c->n)), bb(BLOCK);
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
    hipLaunchKernelGGL(k_pass1_cubic, dim3(blocks_for_groups(c->n)), dim3(BLOCK), 0,
                       c->stream, v, o);
}

void launch_pass2_cubic(lp_ctx* c, const View& v, const double* P, const double* eta,
                        const double* hand, const RhsOut& o)
{
    hipLaunchKernelGGL(k_pass2_cubic, dim3(blocks_for_groups(c->n)), dim3(BLOCK), 0,
                       c->stream, v, P, eta, hand, o);
}

}  // namespace lp
