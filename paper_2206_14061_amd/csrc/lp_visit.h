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

// Along periodic axes a point stands for its copy nearest to the particle
// at (xi, yi).
__device__ __forceinline__ void to_image(const View& v, const GridInfo& g, Pt& p,
                                         double xi, double yi)
{
    if (!v.periodic) return;
    p.x = image_coord(p.x, xi, g.Lx, g.hLx);
    p.y = image_coord(p.y, yi, g.Ly, g.hLy);
}

// Position of real particle j from its 32-byte record.
__device__ __forceinline__ void packed_pos(const View& v, int32_t j, double& x, double& y,
                                          double& z)
{
    const double* r = v.p4 + 4 * (int64_t)j;
    const double2 xy = *reinterpret_cast<const double2*>(r);
    x = xy.x;
    y = xy.y;
    z = r[2];
}

// Point of neighbour-list entry e (a real id, or MBIT | source of a
// potential mirror; the mirror exists while its source is within R of the
// wall, and is placed at (x, y, 2 wall - z)), seen from (xi, yi).
__device__ __forceinline__ Pt list_point(const View& v, const GridInfo& g,
                                         int32_t e, double xi, double yi)
{
    Pt p;
    if (e & MBIT) {
        const int32_t j = e & ~MBIT;
        const int32_t k = v.mirror_of[j];
        p.valid = k >= 0;
        packed_pos(v, j, p.x, p.y, p.z);
        p.z = dsub(dmul(2.0, g.wall), p.z);
        p.id = (int32_t)v.n + k;
        p.src = j;
        p.mirror = true;
    } else {
        p.valid = true;
        packed_pos(v, e, p.x, p.y, p.z);
        p.id = e;
        p.src = e;
        p.mirror = false;
    }
    to_image(v, g, p, xi, yi);
    return p;
}

#ifndef LP_FIT_BATCH
#define LP_FIT_BATCH 4
#endif
// Stencil rows whose loads the fits issue together (by default).
constexpr int FIT_BATCH = LP_FIT_BATCH;

// Registers of one particle's list walk: its position and the fields of
// its system's grid that a list entry needs, copied once so that stores
// made during the walk cannot force the grid table to be read again.
struct Seen {
    double xi, yi, zi;
    double wall2;               // twice the wall height (mirror plane)
    double Lx, hLx, Ly, hLy;    // periodic box, 0 on open axes
};

__device__ __forceinline__ Seen seen_from(const View& v, const GridInfo& g, int64_t i)
{
    Seen s;
    s.xi = v.x[i];
    s.yi = v.y[i];
    s.zi = v.z[i];
    s.wall2 = dmul(2.0, g.wall);
    s.Lx = g.Lx;
    s.hLx = g.hLx;
    s.Ly = g.Ly;
    s.hLy = g.hLy;
    return s;
}

// The points of U list entries (the same points as list_point).  Every
// position load is issued before the first is used, so the U gathers are
// in flight together instead of one latency after another.
template <int U>
__device__ __forceinline__ void gather_list(const View& v, const Seen& s,
                                            const int32_t (&e)[U], Pt (&p)[U])
{
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t j = e[u] & ~MBIT;
        packed_pos(v, j, p[u].x, p[u].y, p[u].z);
        p[u].src = j;
        p[u].id = j;
        p[u].mirror = (e[u] & MBIT) != 0;
        p[u].valid = true;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (p[u].mirror) {
            const int32_t k = v.mirror_of[p[u].src];
            p[u].valid = k >= 0;
            p[u].id = (int32_t)v.n + k;
            p[u].z = dsub(s.wall2, p[u].z);
        }
    }
    if (v.periodic) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            p[u].x = image_coord(p[u].x, s.xi, s.Lx, s.hLx);
            p[u].y = image_coord(p[u].y, s.yi, s.Ly, s.hLy);
        }
    }
}

// Point of a stencil id (real id, or n + k for mirror k), seen from
// (xi, yi).
__device__ __forceinline__ Pt id_point(const View& v, const GridInfo& g,
                                       int32_t id, double xi, double yi)
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
    to_image(v, g, p, xi, yi);
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

// Stencil record of one particle, in registers: kept rows, ghost mask,
// mode and the keep bitmask over its neighbour-list entries.
struct Rec {
    int m, gm, mode;
    uint64_t mask[MASK_WORDS];
};

__device__ __forceinline__ Rec load_rec(const View& v, int64_t i)
{
    Rec r;
    const int64_t n = v.n;
    const int32_t* q = v.rec;
    r.m = q[REC_M * n + i];
    r.gm = q[REC_GM * n + i];
    r.mode = q[REC_MODE * n + i];
#pragma unroll
    for (int w = 0; w < MASK_WORDS; ++w) r.mask[w] = v.kmask[w * n + i];
    return r;
}

// Set bits of a keep mask in ascending order (list indices).
struct MaskWalk {
    static_assert(MASK_WORDS == 4, "keep mask walk assumes four words");
    // the word being walked (entries base, base + 1, ...) and the words
    // after it
    uint64_t cur, b1, b2, b3;
    int base = 0;
    __device__ __forceinline__ explicit MaskWalk(const Rec& r)
        : cur(r.mask[0]), b1(r.mask[1]), b2(r.mask[2]), b3(r.mask[3]) {}
    __device__ __forceinline__ bool any() const { return (cur | b1 | b2 | b3) != 0; }
    // next set bit; the caller pops at most popcount times.  A lane moves
    // to the next word only when its current one is used up (a few times
    // per stencil), so the common pop is one count of trailing zeros.
    __device__ __forceinline__ int pop()
    {
        if (cur == 0) {
            cur = b1;
            b1 = b2;
            b2 = b3;
            b3 = 0;
            base += 64;
            if (cur == 0) {
                cur = b1;
                b1 = b2;
                b2 = 0;
                base += 64;
                if (cur == 0) {
                    cur = b1;
                    b1 = 0;
                    base += 64;
                }
            }
        }
        const int k = base + __builtin_ctzll(cur);
        cur &= cur - 1;
        return k;
    }
};

// Calls f(pt, dx, dy, dz) for every stencil row of real particle i, in
// ascending list order (the ghost rows are not visited: they follow from
// r.gm).  Each lane walks only its own kept entries, so a wave runs as
// many iterations as its largest stencil.  Rows are taken B at a time:
// their list words, then their positions, are loaded together, and the
// calls of f for the batch form one block, so the loads f makes for later
// rows can be issued before the earlier rows are summed.
template <int B = FIT_BATCH, class F>
__device__ __forceinline__ void visit_stencil(const View& v, const GridInfo& g,
                                              int64_t i, const Rec& r, F&& f)
{
    const int64_t n = v.n;
    const Seen s = seen_from(v, g, i);
    const double xi = s.xi, yi = s.yi, zi = s.zi;
    if (r.mode & MODE_SORTED) {
        for (int k = 0; k < r.m; ++k) {
            const Pt p = id_point(v, g, v.hsten[(int64_t)k * n + i], xi, yi);
            f(p, dsub(p.x, xi), dsub(p.y, yi), dsub(p.z, zi));
        }
        return;
    }
    MaskWalk mw(r);
    int t = 0;
    for (; t + B <= r.m; t += B) {
        int32_t e[B];
#pragma unroll
        for (int u = 0; u < B; ++u) e[u] = v.vl[vl_at(n, i, mw.pop())];
        Pt p[B];
        gather_list(v, s, e, p);
#pragma unroll
        for (int u = 0; u < B; ++u)
            f(p[u], dsub(p[u].x, xi), dsub(p[u].y, yi), dsub(p[u].z, zi));
    }
    for (; t < r.m; ++t) {
        const int32_t e[1] = {v.vl[vl_at(n, i, mw.pop())]};
        Pt p[1];
        gather_list(v, s, e, p);
        f(p[0], dsub(p[0].x, xi), dsub(p[0].y, yi), dsub(p[0].z, zi));
    }
}

// Calls f(src, mirror) for every stencil row of real particle i, in the
// order of visit_stencil: the real particle the row's point stands for
// (a mirror's source) and whether it is a mirror.  Reads no positions.
template <int B = 8, class F>
__device__ __forceinline__ void visit_sources(const View& v, int64_t i, const Rec& r, F&& f)
{
    const int64_t n = v.n;
    if (r.mode & MODE_SORTED) {
        for (int k = 0; k < r.m; ++k) {
            const int32_t id = v.hsten[(int64_t)k * n + i];
            if (id < n) f(id, false);
            else f(v.msrc[id - n], true);
        }
        return;
    }
    MaskWalk mw(r);
    int t = 0;
    for (; t + B <= r.m; t += B) {
        int32_t e[B];
#pragma unroll
        for (int u = 0; u < B; ++u) e[u] = v.vl[vl_at(n, i, mw.pop())];
#pragma unroll
        for (int u = 0; u < B; ++u) f(e[u] & ~MBIT, (e[u] & MBIT) != 0);
    }
    for (; t < r.m; ++t) {
        const int32_t e = v.vl[vl_at(n, i, mw.pop())];
        f(e & ~MBIT, (e & MBIT) != 0);
    }
}

// visit_stencil for a particle of a staged tile (not on the sorted path):
// the fields of the tile's list sources sit in LDS in slot order, and a
// row's point is read from there through the slot word of its list entry.
// The Pt handed to f carries the slot in `src` (and no id).  Rows come in
// the same order as from visit_stencil.
template <int B, class F>
__device__ __forceinline__ void visit_staged(const View& v, const Seen& s, int64_t i,
                                             const Rec& r, const double* sx,
                                             const double* sy, const double* sz, F&& f)
{
    const int64_t n = v.n;
    auto row = [&](uint32_t word) {
        Pt p;
        const int q = (int)(word & (SLOT_MIRROR - 1u));
        p.mirror = (word & SLOT_MIRROR) != 0u;
        p.valid = true;
        p.src = q;
        p.id = -1;
        p.x = sx[q];
        p.y = sy[q];
        p.z = p.mirror ? dsub(s.wall2, sz[q]) : sz[q];
        if (v.periodic) {
            p.x = image_coord(p.x, s.xi, s.Lx, s.hLx);
            p.y = image_coord(p.y, s.yi, s.Ly, s.hLy);
        }
        f(p, dsub(p.x, s.xi), dsub(p.y, s.yi), dsub(p.z, s.zi));
    };
    MaskWalk mw(r);
    int t = 0;
    for (; t + B <= r.m; t += B) {
        uint32_t w[B];
#pragma unroll
        for (int u = 0; u < B; ++u) w[u] = v.vs[(int64_t)mw.pop() * n + i];
#pragma unroll
        for (int u = 0; u < B; ++u) row(w[u]);
    }
    for (; t < r.m; ++t) row(v.vs[(int64_t)mw.pop() * n + i]);
}

// visit_staged with the rows of particle i spread over LPP adjacent lanes:
// lane `sub` takes the kept rows sub, sub + LPP, sub + 2 LPP, ... (B of
// them loaded together), in the order of visit_staged.
template <int B, int LPP, class F>
__device__ __forceinline__ void visit_staged_sub(const View& v, const Seen& s, int64_t i,
                                                 const Rec& r, int sub, const double* sx,
                                                 const double* sy, const double* sz, F&& f)
{
    const int64_t n = v.n;
    auto row = [&](uint32_t word) {
        Pt p;
        const int q = (int)(word & (SLOT_MIRROR - 1u));
        p.mirror = (word & SLOT_MIRROR) != 0u;
        p.valid = true;
        p.src = q;
        p.id = -1;
        p.x = sx[q];
        p.y = sy[q];
        p.z = p.mirror ? dsub(s.wall2, sz[q]) : sz[q];
        if (v.periodic) {
            p.x = image_coord(p.x, s.xi, s.Lx, s.hLx);
            p.y = image_coord(p.y, s.yi, s.Ly, s.hLy);
        }
        f(p, dsub(p.x, s.xi), dsub(p.y, s.yi), dsub(p.z, s.zi));
    };
    MaskWalk mw(r);
    // this lane's rows; the walk skips the other lanes' rows
    const int mine = sub < r.m ? (r.m - sub + LPP - 1) / LPP : 0;
    for (int q = 0; q < sub && mw.any(); ++q) mw.pop();
    auto next = [&]() {
        const int k = mw.pop();
#pragma unroll
        for (int q = 1; q < LPP; ++q)
            if (mw.any()) mw.pop();
        return k;
    };
    int t = 0;
    for (; t + B <= mine; t += B) {
        uint32_t w[B];
#pragma unroll
        for (int u = 0; u < B; ++u) w[u] = v.vs[(int64_t)next() * n + i];
#pragma unroll
        for (int u = 0; u < B; ++u) row(w[u]);
    }
    for (; t < mine; ++t) row(v.vs[(int64_t)next() * n + i]);
}

// visit_stencil with the rows of particle i spread over LPP adjacent
// lanes: lane `sub` takes kept rows sub, sub + LPP, sub + 2 LPP, ...
template <int LPP, class F>
__device__ __forceinline__ void visit_stencil_sub(const View& v, const GridInfo& g,
                                                  int64_t i, const Rec& r, int sub, F&& f)
{
    if (LPP == 1) {
        visit_stencil(v, g, i, r, f);
        return;
    }
    const int64_t n = v.n;
    const double xi = v.x[i], yi = v.y[i], zi = v.z[i];
    if (r.mode & MODE_SORTED) {
        for (int k = sub; k < r.m; k += LPP) {
            const Pt p = id_point(v, g, v.hsten[(int64_t)k * n + i], xi, yi);
            f(p, dsub(p.x, xi), dsub(p.y, yi), dsub(p.z, zi));
        }
        return;
    }
    MaskWalk mw(r);
    for (int t = 0; t < sub && t < r.m; ++t) mw.pop();
    for (int t = sub; t < r.m; t += LPP) {
        const int k = mw.pop();
        const Pt p = list_point(v, g, v.vl[vl_at(n, i, k)], xi, yi);
        f(p, dsub(p.x, xi), dsub(p.y, yi), dsub(p.z, zi));
        for (int u = 1; u < LPP && t + u < r.m; ++u) mw.pop();
    }
}

// sum of x over the LPP adjacent lanes of a particle (the same value in
// every one of them: the butterfly adds the same operands in each lane)
template <int LPP, class T>
__device__ __forceinline__ T lane_sum(T x)
{
#pragma unroll
    for (int off = 1; off < LPP; off <<= 1) x += __shfl_xor(x, off);
    return x;
}

}  // namespace lp
