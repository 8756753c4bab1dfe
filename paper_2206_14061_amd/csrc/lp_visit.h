// Iteration over the exact stencil of a particle from its neighbour list
// (with skin) and its stencil record.  Shared by the selection, export and
// fit kernels so that every pass keeps exactly the same rows.
#pragma once

#include "lp_internal.h"

namespace lp {

struct Pt {
    double x, y, z;     // position (mirrors: reflected source)
    int32_t id;         // real id, or n + k for mirror k
    int32_t src;        // real particle carrying the state
    bool mirror;
    bool valid;
};

// Point of neighbour-list entry e (a real id, or MBIT | source of a
// potential mirror; the mirror exists while its source is within R of the
// wall, and is placed at (x, y, 2 wall - z)).
__device__ __forceinline__ Pt list_point(const View& v, const GridInfo& g,
                                         int32_t e)
{
    Pt p;
    if (e & MBIT) {
        const int32_t j = e & ~MBIT;
        const int32_t k = v.mirror_of[j];
        p.valid = k >= 0;
        p.x = v.x[j];
        p.y = v.y[j];
        p.z = dsub(dmul(2.0, g.wall), v.z[j]);
        p.id = (int32_t)v.n + k;
        p.src = j;
        p.mirror = true;
    } else {
        p.valid = true;
        p.x = v.x[e];
        p.y = v.y[e];
        p.z = v.z[e];
        p.id = e;
        p.src = e;
        p.mirror = false;
    }
    return p;
}

// Point of a stencil id (real id, or n + k for mirror k).
__device__ __forceinline__ Pt id_point(const View& v, const GridInfo& g,
                                       int32_t id)
{
    Pt p;
    p.valid = true;
    p.id = id;
    if (id < v.n) {
        p.x = v.x[id];
        p.y = v.y[id];
        p.z = v.z[id];
        p.src = id;
        p.mirror = false;
    } else {
        const int32_t j = v.msrc[id - v.n];
        p.x = v.x[j];
        p.y = v.y[j];
        p.z = dsub(dmul(2.0, g.wall), v.z[j]);
        p.src = j;
        p.mirror = true;
    }
    return p;
}

__device__ __forceinline__ bool key_less(double ra, int32_t ia, double rb,
                                         int32_t ib)
{
    return ra < rb || (ra == rb && ia < ib);
}

__device__ __forceinline__ int octant_of(double dx, double dy, double dz)
{
    return (dx >= 0.0 ? 1 : 0) + (dy >= 0.0 ? 2 : 0) + (dz >= 0.0 ? 4 : 0);
}

// bucket of r^2 in the selection histogram: floor(r2 * scale), clamped
__device__ __forceinline__ int bucket_of(double r2, double scale)
{
    const int b = (int)dmul(r2, scale);
    return b > HIST_BUCKETS - 1 ? HIST_BUCKETS - 1 : b;
}

// sub-bucket of r^2 inside bucket b (monotone in r^2)
__device__ __forceinline__ int sub_of(double r2, double scale, int b)
{
    const int sb = (int)dmul(dsub(dmul(r2, scale), (double)b), (double)HIST_BUCKETS);
    return sb < 0 ? 0 : (sb > HIST_BUCKETS - 1 ? HIST_BUCKETS - 1 : sb);
}

// Stencil record of one particle, in registers.  Octant-firsts and the
// kept members of the cut sub-bucket are list indices (-1 when absent).
struct Rec {
    int m, gm, mode, b, s;
    int32_t first[8];
    int32_t cut[LIST_CAP];
};

__device__ __forceinline__ Rec load_rec(const View& v, int64_t i)
{
    Rec r;
    const int64_t n = v.n;
    const int32_t* q = v.rec;
    r.m = q[REC_M * n + i];
    r.gm = q[REC_GM * n + i];
    r.mode = q[REC_MODE * n + i];
    r.b = q[REC_B * n + i];
    r.s = q[REC_S * n + i];
#pragma unroll
    for (int o = 0; o < 8; ++o) r.first[o] = q[(REC_FIRST + o) * n + i];
#pragma unroll
    for (int o = 0; o < LIST_CAP; ++o) r.cut[o] = q[(REC_CUT + o) * n + i];
    return r;
}

// Whether list entry k, a candidate with key r2, belongs to the stencil.
__device__ __forceinline__ bool keep_entry(const Rec& r, int k, double r2,
                                           double scale)
{
    if (r.mode & MODE_ALL) return true;
    bool f = false;
#pragma unroll
    for (int o = 0; o < 8; ++o) f = f || (r.first[o] == k);
    if (f) return true;
    const int b = bucket_of(r2, scale);
    if (b != r.b) return b < r.b;
    if (!(r.mode & MODE_PARTIAL)) return true;
    const int sb = sub_of(r2, scale, b);
    if (sb != r.s) return sb < r.s;
    if (!(r.mode & MODE_PARTIAL2)) return true;
    bool c = false;
#pragma unroll
    for (int o = 0; o < LIST_CAP; ++o) c = c || (r.cut[o] == k);
    return c;
}

// Calls f(pt, dx, dy, dz) for every stencil row of real particle i (the
// ghost rows are not visited: they follow from r.gm).  cr2 holds the
// candidate key r^2 of every list entry (+inf for non-candidates), as
// stored by the selection.
template <class F>
__device__ __forceinline__ void visit_stencil(const View& v, const GridInfo& g,
                                              const double* __restrict__ cr2,
                                              int64_t i, const Rec& r, F&& f)
{
    const int64_t n = v.n;
    const double xi = v.x[i], yi = v.y[i], zi = v.z[i];
    if (r.mode & MODE_SORTED) {
        for (int k = 0; k < r.m; ++k) {
            const Pt p = id_point(v, g, v.hsten[(int64_t)k * n + i]);
            f(p, dsub(p.x, xi), dsub(p.y, yi), dsub(p.z, zi));
        }
        return;
    }
    const double R2 = g.R2;
    const double scale = (double)HIST_BUCKETS / R2;
    const int cnt = v.vcnt[i];
    for (int k = 0; k < cnt; ++k) {
        const double r2 = cr2[(int64_t)k * n + i];
        if (!(r2 < R2) || !keep_entry(r, k, r2, scale)) continue;
        const Pt p = list_point(v, g, v.vl[(int64_t)k * n + i]);
        f(p, dsub(p.x, xi), dsub(p.y, yi), dsub(p.z, zi));
    }
}

}  // namespace lp
