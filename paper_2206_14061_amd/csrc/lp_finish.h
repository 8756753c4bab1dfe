// Epilogues shared by the fit kernels of every order: the closure and the
// pass-1 hand-off (Sec. 2.2, 2.2.1), the Form E right-hand side of Sec. 2.1
// and the explicit update of Sec. 3.1 steps 8 and 10.
#pragma once

#include "lp_fitcore.h"

namespace lp {

// fields of lp_fit_derivs: k x n values, mirror signs, ghost-zero flags
struct GenericFields {
    const double* f;   // k x n
    int k;
    int32_t msign[8];
    int32_t gzero[8];
};

struct StepOut {
    double* P;
    double* eta;
    double* hand;
    uint8_t* flags;
    double* diag;       // optional 5 x n
    double* coef_u;     // optional 27 x n
};

__device__ __forceinline__ void finish_pass1(const View& v, const lp_params& p,
                                             int64_t i, const double (&c)[27],
                                             const double (&ginv3)[27],
                                             bool has_ginv, uint8_t fl,
                                             const StepOut& o)
{
    const int64_t n = v.n;
    const Closure r = closure(p, v.V[i], c);
    double vis[3];
    visc_terms(c, vis);
    o.P[i] = r.P;
    o.eta[i] = r.eta;
    store_hand(o.hand, n, i, ginv3, has_ginv, r, vis);
    o.flags[i] = (uint8_t)(fl | (r.branch << 1));
    if (o.diag) {
        o.diag[i] = r.P;
        o.diag[n + i] = r.eta;
        o.diag[2 * n + i] = r.I;
        o.diag[3 * n + i] = r.mu;
        o.diag[4 * n + i] = r.gn;
    }
    if (o.coef_u) {
#pragma unroll
        for (int q = 0; q < 27; ++q) o.coef_u[(int64_t)q * n + i] = c[q];
    }
}

struct RhsOut {
    double* acc;        // 3 x n (optional in step mode)
    double* dVdt;       // n (optional in step mode)
    double* grad;       // 6 x n optional
    uint8_t* flags;     // updated with the fallback bit of QR refits
    double* out[7];     // new state (step mode) or nulls
    double dt;
    ErrWord* err;
    Counters* cnt;
    int reflect;        // reflecting wall (step mode)
};

__device__ __forceinline__ void finish_rhs(const View& v, const lp_params& p,
                                           int64_t i, const double* hand,
                                           const double gP[3], const double gE[3],
                                           const RhsOut& o)
{
    const int64_t n = v.n;
    const double V = v.V[i];
    const double eta = hand[0];   // own eta passed through hand[0]
    const double* gd = hand + 1;  // xx yy zz xy xz yz
    const double div = hand[7];
    const double* vis = hand + 8;
    double a[3];
    const double t0 = gd[0] * gE[0] + gd[3] * gE[1] + gd[4] * gE[2];
    const double t1 = gd[3] * gE[0] + gd[1] * gE[1] + gd[5] * gE[2];
    const double t2 = gd[4] * gE[0] + gd[5] * gE[1] + gd[2] * gE[2];
    const double inv_rho = 1.0 / p.rho_s;
    a[0] = V * (-gP[0] + t0 + eta * vis[0]) * inv_rho + p.g[0];
    a[1] = V * (-gP[1] + t1 + eta * vis[1]) * inv_rho + p.g[1];
    a[2] = V * (-gP[2] + t2 + eta * vis[2]) * inv_rho + p.g[2];
    const double dV = V * div;
    if (o.acc) {
        o.acc[i] = a[0];
        o.acc[n + i] = a[1];
        o.acc[2 * n + i] = a[2];
    }
    if (o.dVdt) o.dVdt[i] = dV;
    if (o.grad)
        for (int q = 0; q < 3; ++q) {
            o.grad[(int64_t)q * n + i] = gP[q];
            o.grad[(int64_t)(3 + q) * n + i] = gE[q];
        }
    if (o.out[0]) {
        const double dt = o.dt;
        const double un = v.u[i] + dt * a[0];
        const double vn = v.v[i] + dt * a[1];
        const double wn = v.w[i] + dt * a[2];
        const double xn = wrap_coord(v.x[i] + dt * (0.5 * (v.u[i] + un)), p.box_lo[0],
                                     p.box_len[0]);
        const double yn = wrap_coord(v.y[i] + dt * (0.5 * (v.v[i] + vn)), p.box_lo[1],
                                     p.box_len[1]);
        double zn = v.z[i] + dt * (0.5 * (v.w[i] + wn));
        const double Vn = V + dt * dV;
        double wr = wn;
        if (o.reflect && zn < p.wall_z) {
            zn = dsub(dmul(2.0, p.wall_z), zn);
            wr = -wn;
        }
        o.out[0][i] = xn;
        o.out[1][i] = yn;
        o.out[2][i] = zn;
        o.out[3][i] = un;
        o.out[4][i] = vn;
        o.out[5][i] = wr;
        o.out[6][i] = Vn;
        const bool finite = isfinite(xn) && isfinite(yn) && isfinite(zn) &&
                            isfinite(un) && isfinite(vn) && isfinite(wn) &&
                            isfinite(Vn);
        if (!finite) raise_error(o.err, ERR_NUMERIC, i);
        if (zn < p.wall_z) atomicAdd(&o.cnt->below_wall, 1ull);
    }
}

__device__ __forceinline__ void load_hand_tail(const double* hand, int64_t n,
                                               int64_t i, double eta, double hv[11])
{
    hv[0] = eta;
#pragma unroll
    for (int q = 0; q < 6; ++q) hv[1 + q] = hand[(int64_t)(27 + q) * n + i];
    hv[7] = hand[(int64_t)33 * n + i];
#pragma unroll
    for (int q = 0; q < 3; ++q) hv[8 + q] = hand[(int64_t)(34 + q) * n + i];
}

// cubic (19-unknown) fits, one wavefront per particle (lp_cubic.hip)
void launch_fit3_generic(lp_ctx* c, const View& v, const GenericFields& F, double* coef,
                         uint8_t* flags);
void launch_pass1_cubic(lp_ctx* c, const View& v, const StepOut& o);
void launch_pass2_cubic(lp_ctx* c, const View& v, const double* P, const double* eta,
                        const double* hand, const RhsOut& o);

}  // namespace lp
