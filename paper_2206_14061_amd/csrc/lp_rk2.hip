// Second-order (Heun) time step built from two right-hand-side evaluations
// of the method (Sec. 2.1 with the fits of Sec. 3.1 step 7 and the closure
// of Sec. 2.2): the explicit update of Sec. 3.1 steps 8 and 10 is first
// order in time for u and V; this predictor-corrector pair is the
// second-order time integration the paper names as its next step.
//
//   predictor  s* = s + dt f(s):  x* = x + dt u, u* = u + dt a(s),
//                                 V* = V + dt (V div u)(s)
//   corrector  x' = x + dt (u + u*)/2,  u' = u + dt (a(s) + a(s*))/2,
//              V' = V + dt ((V div u)(s) + (V div u)(s*))/2
//
// Both evaluations use the neighbour list of s; the predictor must stay
// within half the list skin of the positions the list was built for
// (checked on the device, ERR_LIST).
#include "lp_internal.h"

namespace lp {

namespace {

inline unsigned int blocks_for(int64_t n, int per = BLOCK)
{
    return (unsigned int)((n + per - 1) / per);
}

struct S7 {
    const double* p[7];
};

struct O7 {
    double* p[7];
};

__global__ void k_stage(int64_t n, S7 s, const double* acc, const double* dVdt, double dt,
                        O7 o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    o.p[0][i] = s.p[0][i] + dt * s.p[3][i];
    o.p[1][i] = s.p[1][i] + dt * s.p[4][i];
    o.p[2][i] = s.p[2][i] + dt * s.p[5][i];
    o.p[3][i] = s.p[3][i] + dt * acc[i];
    o.p[4][i] = s.p[4][i] + dt * acc[n + i];
    o.p[5][i] = s.p[5][i] + dt * acc[2 * n + i];
    o.p[6][i] = s.p[6][i] + dt * dVdt[i];
}

// the predictor must not leave the list: displacement from the build
// positions below half the skin (d^2 / (skin R)^2 < 1/4)
__global__ void k_stage_check(int64_t n, int n_sys, const int64_t* off,
                              const GridInfo* grid, const double* x, const double* y,
                              const double* z, const double* rx, const double* ry,
                              const double* rz, ErrWord* err)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const GridInfo& g = grid[sys_of(off, n_sys, i)];
    const double dx = image_coord(x[i], rx[i], g.Lx, g.hLx) - rx[i];
    const double dy = image_coord(y[i], ry[i], g.Ly, g.hLy) - ry[i];
    const double dz = z[i] - rz[i];
    const double q = (dx * dx + dy * dy + dz * dz) * g.inv_skin2;
    if (!(q < 0.25)) raise_error(err, ERR_LIST, i);
}

__global__ void k_heun(int64_t n, int n_sys, const int64_t* off, const lp_params* prm,
                       S7 s, S7 s2, const double* acc1, const double* acc2,
                       const double* dV1, const double* dV2, double dt, O7 o,
                       ErrWord* err, Counters* cnt, int reflect)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const lp_params& p = prm[sys_of(off, n_sys, i)];
    const double hdt = 0.5 * dt;
    const double xn = wrap_coord(s.p[0][i] + hdt * (s.p[3][i] + s2.p[3][i]), p.box_lo[0],
                                 p.box_len[0]);
    const double yn = wrap_coord(s.p[1][i] + hdt * (s.p[4][i] + s2.p[4][i]), p.box_lo[1],
                                 p.box_len[1]);
    double zn = s.p[2][i] + hdt * (s.p[5][i] + s2.p[5][i]);
    const double un = s.p[3][i] + hdt * (acc1[i] + acc2[i]);
    const double vn = s.p[4][i] + hdt * (acc1[n + i] + acc2[n + i]);
    double wn = s.p[5][i] + hdt * (acc1[2 * n + i] + acc2[2 * n + i]);
    if (reflect && zn < p.wall_z) {
        zn = dsub(dmul(2.0, p.wall_z), zn);
        wn = -wn;
    }
    const double Vn = s.p[6][i] + hdt * (dV1[i] + dV2[i]);
    o.p[0][i] = xn;
    o.p[1][i] = yn;
    o.p[2][i] = zn;
    o.p[3][i] = un;
    o.p[4][i] = vn;
    o.p[5][i] = wn;
    o.p[6][i] = Vn;
    const bool finite = isfinite(xn) && isfinite(yn) && isfinite(zn) && isfinite(un) &&
                        isfinite(vn) && isfinite(wn) && isfinite(Vn);
    if (!finite) raise_error(err, ERR_NUMERIC, i);
    if (zn < p.wall_z) atomicAdd(&cnt->below_wall, 1ull);
}

}  // namespace

lp_status heun_predictor(lp_ctx* c, double dt)
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (n == 0) return LP_OK;
    hipStream_t st = c->stream;
    S7 s1;
    O7 o2;
    for (int a = 0; a < 7; ++a) {
        s1.p[a] = w.sst[a];
        o2.p[a] = w.sst2[a];
    }
    hipLaunchKernelGGL(k_stage, dim3(blocks_for(n)), dim3(BLOCK), 0, st, n, s1,
                       (const double*)w.acc, (const double*)w.dVdt, dt, o2);
    hipLaunchKernelGGL(k_stage_check, dim3(blocks_for(n)), dim3(BLOCK), 0, st, n,
                       c->n_sys, w.off, w.grid, w.sst2[0], w.sst2[1], w.sst2[2], w.xref[0],
                       w.xref[1], w.xref[2], w.err);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "predictor launch");
}

lp_status step_heun(lp_ctx* c, double dt, double* const out[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (n == 0) return LP_OK;
    lp_status r = heun_predictor(c, dt);
    const double* pred[7];
    for (int a = 0; a < 7; ++a) pred[a] = w.sst2[a];
    if (r == LP_OK) r = stencils_build(c, pred);
    if (r == LP_OK) r = step_rhs(c, pred);
    if (r == LP_OK) r = step_pass2(c, pred, dt, nullptr, w.acc2, w.dVdt2);
    if (r != LP_OK) return r;
    S7 s1, s2;
    O7 oo;
    for (int a = 0; a < 7; ++a) {
        s1.p[a] = w.sst[a];
        s2.p[a] = w.sst2[a];
        oo.p[a] = out[a];
    }
    hipLaunchKernelGGL(k_heun, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, n, c->n_sys,
                       w.off, w.prm, s1, s2, (const double*)w.acc, (const double*)w.acc2,
                       (const double*)w.dVdt, (const double*)w.dVdt2, dt, oo, w.err,
                       w.cnt, c->cfg.wall_reflect);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "corrector launch");
}

}  // namespace lp
