// Morton-sorted cell list and mirror particles (the paper's octree of
// Sec. 3.1 step 4 / Sec. 3.2 replaced by a uniform cell list sorted in
// Z order; mirrors of Sec. 3.1 step 9).
#include <algorithm>
#include <cstring>

#include "lp_internal.h"

namespace lp {

namespace {

// Kernels of the re-sort and list rebuild take a gate word: when it is
// given and zero the kernel does nothing (device-side choice between a
// rebuild and a plain state copy, needed by captured step sequences).
#define LP_GATE(gate) \
    if ((gate) && *(gate) == 0) return

__device__ __forceinline__ unsigned long long ord_enc(double d)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(d);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ double ord_dec(unsigned long long e)
{
    unsigned long long b = (e >> 63) ? (e & 0x7FFFFFFFFFFFFFFFull) : ~e;
    return __longlong_as_double((long long)b);
}

__global__ void k_bbox_init(unsigned long long* bbox, int n_sys, const int32_t* gate)
{
    LP_GATE(gate);
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 6 * n_sys) bbox[t] = (t % 6) < 3 ? ~0ull : 0ull;
}

constexpr int BBOX_CHUNK = 8;

__device__ void bbox_flush(unsigned long long* bbox, int s, const double* lo,
                           const double* hi)
{
    for (int a = 0; a < 3; ++a) {
        atomicMin(&bbox[6 * s + a], ord_enc(lo[a]));
        atomicMax(&bbox[6 * s + 3 + a], ord_enc(hi[a]));
    }
}

// Per-system bounding box of the real particles.
__global__ void k_bbox(int64_t n, int n_sys, const int64_t* off,
                       const double* x, const double* y, const double* z,
                       unsigned long long* bbox, const int32_t* gate)
{
    LP_GATE(gate);
    // block b covers BLOCK x BBOX_CHUNK consecutive particles; thread t
    // takes every BLOCK-th of them from b's start + t (coalesced loads, and
    // increasing indices, so the systems it meets come in order)
    const int64_t b = (int64_t)blockIdx.x * BLOCK * BBOX_CHUNK + threadIdx.x;
    const int lane = threadIdx.x & 63;
    // a block inside one system (the common case): every load of a thread
    // issued before its minima, then one flush per block
    {
        const int64_t b0 = (int64_t)blockIdx.x * BLOCK * BBOX_CHUNK;
        const int64_t b1 = (b0 + BLOCK * BBOX_CHUNK < n ? b0 + BLOCK * BBOX_CHUNK : n) - 1;
        const int s0 = sys_of(off, n_sys, b0);
        if (s0 == sys_of(off, n_sys, b1)) {
            __shared__ double part[6][BLOCK / 64];
            double q[3][BBOX_CHUNK];
#pragma unroll
            for (int k = 0; k < BBOX_CHUNK; ++k) {
                // past n: the first particle of the block again
                const int64_t i = b + (int64_t)k * BLOCK < n ? b + (int64_t)k * BLOCK : b0;
                q[0][k] = x[i];
                q[1][k] = y[i];
                q[2][k] = z[i];
            }
            double m[6];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                m[a] = m[3 + a] = q[a][0];
#pragma unroll
                for (int k = 1; k < BBOX_CHUNK; ++k) {
                    m[a] = fmin(m[a], q[a][k]);
                    m[3 + a] = fmax(m[3 + a], q[a][k]);
                }
            }
            for (int o = 32; o > 0; o >>= 1)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    m[a] = fmin(m[a], __shfl_xor(m[a], o));
                    m[3 + a] = fmax(m[3 + a], __shfl_xor(m[3 + a], o));
                }
            if (lane == 0)
#pragma unroll
                for (int a = 0; a < 6; ++a) part[a][threadIdx.x >> 6] = m[a];
            __syncthreads();
            if (threadIdx.x == 0) {
#pragma unroll
                for (int w = 1; w < BLOCK / 64; ++w)
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        m[a] = fmin(m[a], part[a][w]);
                        m[3 + a] = fmax(m[3 + a], part[3 + a][w]);
                    }
                bbox_flush(bbox, s0, m, m + 3);
            }
            return;
        }
    }
    int cur = -1;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    if (b < n) {
        const int64_t e = b + (int64_t)BLOCK * BBOX_CHUNK;
        for (int64_t i = b; i < e && i < n; i += BLOCK) {
            int s = cur;
            if (s < 0 || i >= off[s + 1]) s = sys_of(off, n_sys, i);
            if (s != cur) {
                if (cur >= 0) bbox_flush(bbox, cur, lo, hi);
                cur = s;
                lo[0] = hi[0] = x[i];
                lo[1] = hi[1] = y[i];
                lo[2] = hi[2] = z[i];
            }
            const double q[3] = {x[i], y[i], z[i]};
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(lo[a], q[a]);
                hi[a] = fmax(hi[a], q[a]);
            }
        }
    }
    // wave-level combine when every lane holds the same system
    const int first = __shfl(cur, 0);
    const unsigned long long same = __ballot(cur == first);
    if (same == ~0ull && first >= 0) {
        for (int off2 = 32; off2 > 0; off2 >>= 1)
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(lo[a], __shfl_xor(lo[a], off2));
                hi[a] = fmax(hi[a], __shfl_xor(hi[a], off2));
            }
        if (lane == 0) bbox_flush(bbox, first, lo, hi);
    } else if (cur >= 0) {
        bbox_flush(bbox, cur, lo, hi);
    }
}

// Grid of each system from its bounding box; totals for the host.  Cell
// edge c = R (1 + skin) (1 + 2^-20) >= the list radius.  With max_bits > 0
// (captured steps, no host check) every edge is scaled up by a common
// factor until each axis needs at most max_bits bits and all cells fit in
// max_cells: any edge at least the list radius finds the same pairs.
__global__ void k_grid(int n_sys, const int64_t* off, const lp_params* prm,
                       double skin, const unsigned long long* bbox,
                       GridInfo* grid, Summary* sum, int max_bits,
                       int64_t max_cells, ErrWord* err, const int32_t* gate)
{
    LP_GATE(gate);
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double scale = 1.0;
    for (int attempt = 0; attempt < 64; ++attempt) {
        int64_t base = 0;
        int bits = 0, bad = 0;
        for (int s = 0; s < n_sys; ++s) {
            const lp_params& p = prm[s];
            GridInfo g;
            g.pbeg = off[s];
            g.pend = off[s + 1];
            g.R = p.R;
            g.R2 = dmul(p.R, p.R);
            g.h = p.h;
            g.inv_h = 1.0 / p.h;
            g.wall = p.wall_z;
            g.Rv = dmul(p.R, 1.0 + skin);
            g.Rv2 = dmul(g.Rv, g.Rv);
            g.inv_skin2 = skin > 0.0 ? 1.0 / ((skin * p.R) * (skin * p.R)) : 0.0;
            const double c = dmul(dmul(g.Rv, 1.0 + 1.0 / 1048576.0), scale);
            g.inv_c = 1.0 / c;
            g.inv_cx = g.inv_cy = g.inv_c;
            g.xlo = p.box_lo[0];
            g.ylo = p.box_lo[1];
            g.Lx = p.box_len[0];
            g.Ly = p.box_len[1];
            g.hLx = 0.5 * g.Lx;
            g.hLy = 0.5 * g.Ly;
            if (g.pend > g.pbeg) {
                double lo[3], hi[3];
                for (int a = 0; a < 3; ++a) {
                    lo[a] = ord_dec(bbox[6 * s + a]);
                    hi[a] = ord_dec(bbox[6 * s + 3 + a]);
                }
                g.x0 = lo[0];
                g.y0 = lo[1];
                const double zl = dsub(p.wall_z, p.R);
                g.z0 = zl < lo[2] ? zl : lo[2];
                const double ex = dmul(dsub(hi[0], g.x0), g.inv_c);
                const double ey = dmul(dsub(hi[1], g.y0), g.inv_c);
                const double ez = dmul(dsub(hi[2], g.z0), g.inv_c);
                if (!(ex < 65535.0 && ey < 65535.0 && ez < 65535.0)) {
                    bad = 1;
                    g.nx = g.ny = g.nz = 1;
                } else {
                    g.nx = (int)ex + 1;
                    g.ny = (int)ey + 1;
                    g.nz = (int)ez + 1;
                }
                // a periodic axis starts at its box and holds floor(L / c)
                // cells of edge L / n (at least c)
                if (g.Lx > 0.0) {
                    const double e = dmul(g.Lx, g.inv_c);
                    if (!(e < 65535.0)) bad = 1;
                    const int np = e < 65535.0 ? (int)e : 1;
                    g.nx = np < 1 ? 1 : np;
                    g.x0 = g.xlo;
                    g.inv_cx = (double)g.nx / g.Lx;
                }
                if (g.Ly > 0.0) {
                    const double e = dmul(g.Ly, g.inv_c);
                    if (!(e < 65535.0)) bad = 1;
                    const int np = e < 65535.0 ? (int)e : 1;
                    g.ny = np < 1 ? 1 : np;
                    g.y0 = g.ylo;
                    g.inv_cy = (double)g.ny / g.Ly;
                }
            } else {
                g.x0 = g.y0 = g.z0 = 0.0;
                g.nx = g.ny = g.nz = 1;
            }
            int m = g.nx > g.ny ? g.nx : g.ny;
            m = m > g.nz ? m : g.nz;
            int b = 0;
            while ((1 << b) < m) ++b;
            bits = b > bits ? b : bits;
            g.cell_base = base;
            g.pad = 0;
            base += (int64_t)g.nx * g.ny * g.nz;
            grid[s] = g;
        }
        const bool fits = !bad && bits <= max_bits && base <= max_cells;
        if (max_bits <= 0 || fits) {
            sum->total_cells = base;
            sum->axis_bits = bits;
            sum->bad = bad;
            return;
        }
        if (attempt == 63) {
            // cannot happen for any state that fits in memory; keep every
            // later kernel in bounds and report it
            for (int s2 = 0; s2 < n_sys; ++s2) {
                grid[s2].nx = grid[s2].ny = grid[s2].nz = 1;
                grid[s2].cell_base = s2;
            }
            sum->total_cells = n_sys;
            sum->axis_bits = 0;
            sum->bad = 1;
            raise_error(err, ERR_CAPACITY, 0);
            return;
        }
        scale *= 1.25;
    }
}

__device__ __forceinline__ void cell_of(const GridInfo& g, double x, double y,
                                        double z, int& cx, int& cy, int& cz)
{
    const double xw = wrap_coord(x, g.xlo, g.Lx), yw = wrap_coord(y, g.ylo, g.Ly);
    int ix = (int)dmul(dsub(xw, g.x0), g.inv_cx);
    int iy = (int)dmul(dsub(yw, g.y0), g.inv_cy);
    int iz = (int)dmul(dsub(z, g.z0), g.inv_c);
    cx = ix < 0 ? 0 : (ix >= g.nx ? g.nx - 1 : ix);
    cy = iy < 0 ? 0 : (iy >= g.ny ? g.ny - 1 : iy);
    cz = iz < 0 ? 0 : (iz >= g.nz ? g.nz - 1 : iz);
}

// Sort keys (system, Morton code of the cell) and identity values.
__global__ void k_keys(int64_t n, int n_sys, const int64_t* off,
                       const GridInfo* grid, const double* x, const double* y,
                       const double* z, int shift_sys,
                       unsigned long long* keys, int32_t* vals, ErrWord* err,
                       const int32_t* gate)
{
    LP_GATE(gate);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = sys_of(off, n_sys, i);
    const GridInfo& g = grid[s];
    int cx, cy, cz;
    cell_of(g, x[i], y[i], z[i], cx, cy, cz);
    keys[i] = ((unsigned long long)s << shift_sys) | morton3(cx, cy, cz);
    vals[i] = (int32_t)i;
    // positions along a periodic axis must lie within one period of the box
    const bool outx = g.Lx > 0.0 && !(x[i] >= dsub(g.xlo, g.Lx) &&
                                      x[i] < dadd(g.xlo, dmul(2.0, g.Lx)));
    const bool outy = g.Ly > 0.0 && !(y[i] >= dsub(g.ylo, g.Ly) &&
                                      y[i] < dadd(g.ylo, dmul(2.0, g.Ly)));
    if (outx || outy) raise_error(err, ERR_BOX, i);
}

// ---- stable LSD radix sort, digits of up to RADIX_MAX_BITS bits ---------

static_assert(RADIX_MAX_DIGITS == 2 * BLOCK, "each thread owns two digits");

__global__ void k_radix_hist(const unsigned long long* keys, int64_t n,
                             int shift, int dbits, uint32_t* hist, int64_t nblk,
                             const int32_t* gate)
{
    LP_GATE(gate);
    __shared__ uint32_t h[RADIX_MAX_DIGITS];
    const int t = threadIdx.x;
    const unsigned long long mask = (1ull << dbits) - 1ull;
    h[t] = 0;
    h[t + BLOCK] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * BLOCK + t;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & mask], 1u);
    }
    __syncthreads();
    const int nd = 1 << dbits;
    if (t < nd) hist[(int64_t)t * nblk + blockIdx.x] = h[t];
    if (t + BLOCK < nd) hist[(int64_t)(t + BLOCK) * nblk + blockIdx.x] = h[t + BLOCK];
}

// Exclusive scan in place of a uint32 array (single block of 1024).
// In-place exclusive prefix sum of a[0, total) by one block of 1024
// threads, SCAN_TILE values at a time: a tile is loaded coalesced into LDS
// (padded against bank conflicts), each thread scans SCAN_PER consecutive
// values, the block scans the thread sums, and the tile is written back
// coalesced with the running total of the tiles before it added.
constexpr int SCAN_THREADS = 1024, SCAN_PER = 8, SCAN_TILE = SCAN_THREADS * SCAN_PER;

__device__ __forceinline__ int scan_pad(int q) { return q + (q >> 5); }

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_u32(uint32_t* a, int64_t total,
                                                           const int32_t* gate)
{
    LP_GATE(gate);
    __shared__ uint32_t buf[SCAN_TILE + SCAN_TILE / 32];
    __shared__ uint32_t wsum[SCAN_THREADS / 64];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t carry = 0;
    for (int64_t base = 0; base < total; base += SCAN_TILE) {
        uint32_t v[SCAN_PER];
#pragma unroll
        for (int r = 0; r < SCAN_PER; ++r) {
            const int64_t q = base + t + (int64_t)r * SCAN_THREADS;
            v[r] = q < total ? a[q] : 0u;
        }
#pragma unroll
        for (int r = 0; r < SCAN_PER; ++r) buf[scan_pad(t + r * SCAN_THREADS)] = v[r];
        __syncthreads();
        uint32_t loc[SCAN_PER];
        uint32_t sum = 0;
#pragma unroll
        for (int r = 0; r < SCAN_PER; ++r) {
            loc[r] = buf[scan_pad(t * SCAN_PER + r)];
            sum += loc[r];
        }
        // exclusive scan of the thread sums: within each wave, then across
        uint32_t inc = sum;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(inc, d);
            if (lane >= d) inc += o;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        uint32_t pre = carry + inc - sum, tile_total = 0;
        for (int w = 0; w < SCAN_THREADS / 64; ++w) {
            if (w < wave) pre += wsum[w];
            tile_total += wsum[w];
        }
#pragma unroll
        for (int r = 0; r < SCAN_PER; ++r) {
            buf[scan_pad(t * SCAN_PER + r)] = pre;
            pre += loc[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SCAN_PER; ++r) {
            const int ql = t + r * SCAN_THREADS;
            const int64_t q = base + ql;
            if (q < total) a[q] = buf[scan_pad(ql)];
        }
        carry += tile_total;
        __syncthreads();   // buf and wsum are reused by the next tile
    }
}

__global__ void k_radix_scatter(const unsigned long long* kin,
                                const int32_t* vin, unsigned long long* kout,
                                int32_t* vout, int64_t n, int shift, int dbits,
                                const uint32_t* hist, int64_t nblk, const int32_t* gate)
{
    LP_GATE(gate);
    __shared__ uint32_t base[RADIX_MAX_DIGITS];
    __shared__ uint32_t run[RADIX_MAX_DIGITS];
    __shared__ uint32_t wcnt[BLOCK / 64][RADIX_MAX_DIGITS];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    const int nd = 1 << dbits;
    const uint32_t mask = (uint32_t)nd - 1u;
    // thread t owns digits t and t + BLOCK
    for (int q = 0; q < 2; ++q) {
        const int d = t + q * BLOCK;
        base[d] = d < nd ? hist[(int64_t)d * nblk + blockIdx.x] : 0u;
        run[d] = 0;
        for (int w = 0; w < BLOCK / 64; ++w) wcnt[w][d] = 0;
    }
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t tb = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = tb + (int64_t)r * BLOCK + t;
        const bool valid = i < n;
        const unsigned long long key = valid ? kin[i] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        // lanes holding the same digit: match the digit bit by bit
        unsigned long long peers = __ballot(valid);
        for (int bit = 0; bit < dbits; ++bit) {
            const bool on = (d >> bit) & 1u;
            const unsigned long long bal = __ballot(on);
            peers &= on ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[d] + run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        for (int q = 0; q < 2; ++q) {
            const int dd = t + q * BLOCK;
            uint32_t add = 0;
            for (int w = 0; w < BLOCK / 64; ++w) {
                add += wcnt[w][dd];
                wcnt[w][dd] = 0;
            }
            run[dd] += add;
        }
        __syncthreads();
    }
}

struct State7 {
    const double* a[7];
};
struct Dest7 {
    double* a[7];
};

// The state in sorted order (perm[new] = old; perm null: the same order);
// for a rebuild (rx not null) the positions again as the reference of the
// next displacement check; the positions' 32-byte records (p4, optional);
// and the caller's particle ids (ids, optional) into ids_tmp.
__global__ void k_gather7(int64_t n, const int32_t* perm, State7 in, Dest7 out,
                          double* rx, double* ry, double* rz, double* p4,
                          const int32_t* ids, int32_t* ids_tmp, const int32_t* gate)
{
    LP_GATE(gate);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm ? perm[i] : i;
    double v[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) v[a] = in.a[a][j];
#pragma unroll
    for (int a = 0; a < 7; ++a) out.a[a][i] = v[a];
    if (rx) {
        rx[i] = v[0];
        ry[i] = v[1];
        rz[i] = v[2];
    }
    if (p4) {
        // the positions' records, which the list build and the selection read
        double2* r = reinterpret_cast<double2*>(p4 + 4 * i);
        r[0] = make_double2(v[0], v[1]);
        r[1] = make_double2(v[2], 0.0);
    }
    if (ids) ids_tmp[i] = ids[j];
}

__global__ void k_copy_i32(int64_t n, const int32_t* a, int32_t* b, const int32_t* gate)
{
    LP_GATE(gate);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_copy_f64(int64_t n, const double* a, double* b, const int32_t* gate)
{
    LP_GATE(gate);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// a[0..count) = b[0..count) = v, with count = *count_dev when given
// (grid-stride)
__global__ void k_fill2_i32(int64_t n, int32_t* a, int32_t* b, int32_t v,
                            const int64_t* count_dev, const int32_t* gate)
{
    LP_GATE(gate);
    int64_t m = n;
    if (count_dev) m = *count_dev < n ? *count_dev : n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x) {
        a[i] = v;
        b[i] = v;
    }
}

// Cell start/end from sorted keys; positions give the linear cell index.
__global__ void k_cell_bounds(int64_t cnt, int n_sys, const int64_t* off,
                              const GridInfo* grid,
                              const unsigned long long* keys,
                              const double* x, const double* y,
                              const double* z, int32_t* cs, int32_t* ce,
                              const int32_t* ids_tmp, int32_t* ids, const int32_t* gate)
{
    LP_GATE(gate);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    // the ids k_gather7 gathered (every gather has completed)
    if (ids) ids[i] = ids_tmp[i];
    const unsigned long long k = keys[i];
    const bool first = (i == 0) || keys[i - 1] != k;
    const bool last = (i == cnt - 1) || keys[i + 1] != k;
    if (!first && !last) return;
    const int s = sys_of(off, n_sys, i);
    const GridInfo& g = grid[s];
    int cx, cy, cz;
    cell_of(g, x[i], y[i], z[i], cx, cy, cz);
    const int64_t c = g.cell_base + cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz);
    if (first) cs[c] = (int32_t)i;
    if (last) ce[c] = (int32_t)(i + 1);
}

__global__ void k_iota(int64_t n, int32_t* p, const int32_t* gate)
{
    LP_GATE(gate);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

__global__ void k_disp_init(Summary* sum) { sum->disp = DISP_ZERO; }

// blocks of the state copy with the displacement check (one maximum per
// block goes to the summary; 256 to 1,024 time alike, 2,048 slower)
constexpr unsigned COPY_BLOCKS = 512u;

// (displacement since the last build / skin)^2 of one particle; infinite
// for non-finite positions, which force a rebuild
__device__ __forceinline__ double disp_ratio(const GridInfo& g, double x, double y, double z,
                                             double rx, double ry, double rz)
{
    const double dx = image_coord(x, rx, g.Lx, g.hLx) - rx;
    const double dy = image_coord(y, ry, g.Ly, g.hLy) - ry;
    const double dz = z - rz;
    const double d2 = dx * dx + dy * dy + dz * dz;
    double q = g.inv_skin2 > 0.0 ? d2 * g.inv_skin2 : (d2 > 0.0 ? INFINITY : 0.0);
    if (!(q == q)) q = INFINITY;
    return q;
}

__device__ __forceinline__ void disp_block_max(double r, double* part, Summary* sum)
{
    for (int d = 32; d > 0; d >>= 1) r = fmax(r, __shfl_xor(r, d));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < BLOCK / 64; ++w) r = fmax(r, part[w]);
        atomicMax(&sum->disp, ord_enc(r));
    }
}

// k_copy_disp on pairs of particles: 16-byte loads and stores of every
// array (all 16-byte aligned), half the memory instructions; an odd last
// particle is taken by one thread.
__global__ __launch_bounds__(BLOCK) void k_copy_disp2(int64_t n, int n_sys,
                                                      const int64_t* off,
                                                      const GridInfo* grid, State7 st,
                                                      Dest7 dst, const double* rx,
                                                      const double* ry, const double* rz,
                                                      double* p4, Summary* sum)
{
    __shared__ double part[BLOCK / 64];
    double r = 0.0;
    const int64_t np = n >> 1;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < np;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = 2 * j;
        // every load before the first store (the compiler cannot move
        // loads above stores to arrays that might alias them)
        double2 f[7];
#pragma unroll
        for (int a = 0; a < 7; ++a) f[a] = reinterpret_cast<const double2*>(st.a[a])[j];
        const double2 qx = reinterpret_cast<const double2*>(rx)[j];
        const double2 qy = reinterpret_cast<const double2*>(ry)[j];
        const double2 qz = reinterpret_cast<const double2*>(rz)[j];
#pragma unroll
        for (int a = 0; a < 7; ++a) reinterpret_cast<double2*>(dst.a[a])[j] = f[a];
        double2* rec = reinterpret_cast<double2*>(p4 + 4 * i);
        rec[0] = make_double2(f[0].x, f[1].x);
        rec[1] = make_double2(f[2].x, 0.0);
        rec[2] = make_double2(f[0].y, f[1].y);
        rec[3] = make_double2(f[2].y, 0.0);
        r = fmax(r, disp_ratio(grid[sys_of(off, n_sys, i)], f[0].x, f[1].x, f[2].x, qx.x,
                               qy.x, qz.x));
        r = fmax(r, disp_ratio(grid[sys_of(off, n_sys, i + 1)], f[0].y, f[1].y, f[2].y,
                               qx.y, qy.y, qz.y));
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t i = n - 1;
        double f[7];
#pragma unroll
        for (int a = 0; a < 7; ++a) f[a] = st.a[a][i];
#pragma unroll
        for (int a = 0; a < 7; ++a) dst.a[a][i] = f[a];
        double2* rec = reinterpret_cast<double2*>(p4 + 4 * i);
        rec[0] = make_double2(f[0], f[1]);
        rec[1] = make_double2(f[2], 0.0);
        r = fmax(r, disp_ratio(grid[sys_of(off, n_sys, i)], f[0], f[1], f[2], rx[i], ry[i],
                               rz[i]));
    }
    disp_block_max(r, part, sum);
}

// k_disp fused with the copy of the seven state arrays into the working
// state (one pass over the state).
// The positions also go to their 32-byte records (p4), which the
// selection and the list build read.
__global__ __launch_bounds__(BLOCK) void k_copy_disp(int64_t n, int n_sys,
                                                     const int64_t* off,
                                                     const GridInfo* grid, State7 st,
                                                     Dest7 dst, const double* rx,
                                                     const double* ry, const double* rz,
                                                     double* p4, Summary* sum)
{
    __shared__ double part[BLOCK / 64];
    double r = 0.0;
    // grid-stride over particles (a few hundred blocks, so that few blocks
    // contend for the one atomic below)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double f[7];
#pragma unroll
        for (int a = 0; a < 7; ++a) f[a] = st.a[a][i];
#pragma unroll
        for (int a = 0; a < 7; ++a) dst.a[a][i] = f[a];
        double2* rec = reinterpret_cast<double2*>(p4 + 4 * i);
        rec[0] = make_double2(f[0], f[1]);
        rec[1] = make_double2(f[2], 0.0);
        r = fmax(r, disp_ratio(grid[sys_of(off, n_sys, i)], f[0], f[1], f[2], rx[i], ry[i],
                               rz[i]));
    }
    disp_block_max(r, part, sum);
}

inline unsigned int blocks_for(int64_t n, int per = BLOCK)
{
    return (unsigned int)((n + per - 1) / per);
}

// Sorts (keys, vals) of length cnt over `bits` bits; returns the buffers
// holding the result through kr / vr.
void radix_sort(lp_ctx* c, int64_t cnt, int bits, unsigned long long*& kr,
                int32_t*& vr, const int32_t* gate)
{
    Work& w = c->w;
    unsigned long long* kin = w.keys0;
    unsigned long long* kout = w.keys1;
    int32_t* vin = w.vals0;
    int32_t* vout = w.vals1;
    const int64_t nblk = (cnt + SORT_TILE - 1) / SORT_TILE;
    // the fewest passes of at most RADIX_MAX_BITS bits, digits of equal
    // width (18 bits: two passes of 9)
    const int passes = bits <= 0 ? 0 : (bits + RADIX_MAX_BITS - 1) / RADIX_MAX_BITS;
    const int dbits = passes > 0 ? (bits + passes - 1) / passes : 0;
    for (int p = 0; p < passes && cnt > 0; ++p) {
        const int shift = dbits * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(BLOCK), 0,
                           c->stream, kin, cnt, shift, dbits, w.hist, nblk, gate);
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(SCAN_THREADS), 0, c->stream,
                           w.hist, (int64_t)(1 << dbits) * nblk, gate);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(BLOCK),
                           0, c->stream, kin, vin, kout, vout, cnt, shift, dbits,
                           w.hist, nblk, gate);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    kr = kin;
    vr = vin;
}

// Rebuild decision of a captured step: gate[0] = rebuild (re-sort and
// rebuild the list), when some particle has moved 0.49 skin R since the
// last build (or always when `force`).
__global__ void k_decide(Summary* sum, int32_t* gate, Counters* cnt, int force,
                         unsigned long long* bbox, int n_sys)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double r = ord_dec(sum->disp);
    const bool rebuild = force || !(sqrt(r) < 0.49);
    gate[0] = rebuild ? 1 : 0;
    // the next step's displacement check starts from zero
    sum->disp = DISP_ZERO;
    if (!rebuild) return;
    atomicAdd(&cnt->rebuilds, 1ull);
    // empty bounding boxes for the rebuild's k_bbox (as k_bbox_init)
    for (int q = 0; q < 6 * n_sys; ++q) bbox[q] = (q % 6) < 3 ? ~0ull : 0ull;
}

__global__ void k_gather_i32(int64_t n, const int32_t* perm, const int32_t* a,
                             int32_t* b, const int32_t* gate)
{
    LP_GATE(gate);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[perm[i]];
}

// Re-sort + cell tables (+ list): eagerly with one host synchronisation for
// the grid sizes (gate == nullptr), or entirely on the device behind a
// gate with the grid held to `dev_bits` bits per axis.
lp_status rebuild(lp_ctx* c, double* const st[7], int32_t* perm_out, int32_t* ids,
                  const int32_t* gate, int dev_bits)
{
    Work& w = c->w;
    const int64_t n = c->n;
    const int ns = c->n_sys;
    hipStream_t s = c->stream;
    const bool dev = gate != nullptr;
    if (!dev) {
        c->cells_ok = false;
        c->stencils_ok = false;
        c->list_ok = false;
    }
    // (a captured step's k_decide empties the boxes when it decides to
    // rebuild)
    if (!dev)
        hipLaunchKernelGGL(k_bbox_init, dim3(blocks_for(6 * ns)), dim3(BLOCK), 0,
                           s, w.bbox, ns, gate);
    if (n > 0)
        hipLaunchKernelGGL(k_bbox, dim3(blocks_for((n + BBOX_CHUNK - 1) / BBOX_CHUNK)),
                           dim3(BLOCK), 0, s, n, ns, w.off, st[0], st[1], st[2],
                           w.bbox, gate);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(64), 0, s, ns, w.off, w.prm,
                       c->cfg.skin, w.bbox, w.grid, w.summary, dev ? dev_bits : 0,
                       w.cells_max, w.err, gate);
    int axis_bits = dev_bits;
    if (!dev) {
        hipError_t e = hipMemcpyAsync(w.h_summary, w.summary, sizeof(Summary),
                                      hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(c, e, "grid summary");
        const Summary sm = *w.h_summary;
        if (sm.bad) {
            c->err = "a system spans more than 65535 cells along one axis";
            return LP_E_CAPACITY;
        }
        if (sm.total_cells > w.cells_max) {
            c->err = "cell tables need " + std::to_string(sm.total_cells) +
                     " cells, reserved " + std::to_string(w.cells_max);
            return LP_E_CAPACITY;
        }
        c->axis_bits = axis_bits = sm.axis_bits;
        c->total_cells = sm.total_cells;
    }
    int sys_bits = 0;
    while ((1 << sys_bits) < ns) ++sys_bits;
    const int shift_sys = 3 * axis_bits;
    const int bits = shift_sys + sys_bits;

    unsigned long long* kr = nullptr;
    int32_t* vr = nullptr;
    if (n > 0) {
        hipLaunchKernelGGL(k_keys, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, ns,
                           w.off, w.grid, st[0], st[1], st[2], shift_sys, w.keys0,
                           w.vals0, w.err, gate);
        radix_sort(c, n, bits, kr, vr, gate);
        State7 s7;
        Dest7 d7;
        for (int a = 0; a < 7; ++a) {
            s7.a[a] = st[a];
            d7.a[a] = w.sst[a];
        }
        hipLaunchKernelGGL(k_gather7, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, vr, s7,
                           d7, w.xref[0], w.xref[1], w.xref[2], w.p4, ids, w.ids_tmp,
                           gate);
        if (perm_out)
            hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(n)), dim3(BLOCK), 0, s,
                               n, vr, perm_out, gate);
    }
    // cell tables: the whole used range (read on the device in captured
    // steps)
    const int64_t tc = dev ? w.cells_max : c->total_cells;
    const int64_t* tdev = dev ? &w.summary->total_cells : nullptr;
    const unsigned fb = std::min(blocks_for(tc), 8192u);
    hipLaunchKernelGGL(k_fill2_i32, dim3(fb), dim3(BLOCK), 0, s, tc, w.cs, w.ce, 0, tdev,
                       gate);
    if (n > 0)
        hipLaunchKernelGGL(k_cell_bounds, dim3(blocks_for(n)), dim3(BLOCK), 0, s,
                           n, ns, w.off, w.grid, kr, w.sst[0], w.sst[1], w.sst[2],
                           w.cs, w.ce, w.ids_tmp, ids, gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "cell build launch");
    if (!dev) c->cells_ok = true;
    return list_build(c, gate);
}

}  // namespace

lp_status cells_build(lp_ctx* c, double* const st[7], int32_t* perm_out)
{
    return rebuild(c, st, perm_out, nullptr, nullptr, 0);
}

lp_status cells_build_device(lp_ctx* c, double* const st[7], int32_t* ids,
                             const int32_t* gate, int bits)
{
    return rebuild(c, st, nullptr, ids, gate, bits);
}

lp_status state_copy(lp_ctx* c, double* const st[7], int32_t* perm_out,
                     const int32_t* gate, bool arrays)
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (n > 0) {
        for (int a = 0; a < 7 && arrays; ++a)
            hipLaunchKernelGGL(k_copy_f64, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, n, st[a], w.sst[a], gate);
        if (perm_out)
            hipLaunchKernelGGL(k_iota, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, n, perm_out, gate);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "state copy");
}

lp_status permute_ids(lp_ctx* c, const int32_t* perm, int32_t* ids)
{
    const int64_t n = c->n;
    if (n > 0) {
        hipLaunchKernelGGL(k_gather_i32, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream,
                           n, perm, ids, c->w.ids_tmp, nullptr);
        hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream,
                           n, c->w.ids_tmp, ids, nullptr);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "id permutation");
}

lp_status state_gather(lp_ctx* c, const double* const st[7], const int32_t* perm)
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (n > 0)
    {
        State7 s7;
        Dest7 d7;
        for (int a = 0; a < 7; ++a) {
            s7.a[a] = st[a];
            d7.a[a] = w.sst[a];
        }
        hipLaunchKernelGGL(k_gather7, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream, n,
                           perm, s7, d7, nullptr, nullptr, nullptr, w.p4, nullptr,
                           nullptr, nullptr);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "state gather");
}

// The state copy with the displacement check (k_copy_disp, or its
// paired form when every array is 16-byte aligned).
static void launch_copy_disp(lp_ctx* c, const double* const st[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    State7 s7;
    Dest7 d7;
    bool al = (reinterpret_cast<uintptr_t>(w.p4) & 15u) == 0;
    for (int a = 0; a < 7; ++a) {
        s7.a[a] = st[a];
        d7.a[a] = w.sst[a];
        al = al && (reinterpret_cast<uintptr_t>(st[a]) & 15u) == 0 &&
             (reinterpret_cast<uintptr_t>(w.sst[a]) & 15u) == 0;
    }
    for (int a = 0; a < 3; ++a) al = al && (reinterpret_cast<uintptr_t>(w.xref[a]) & 15u) == 0;
    if (al)
        hipLaunchKernelGGL(k_copy_disp2, dim3(std::min(blocks_for((n + 1) / 2), COPY_BLOCKS)),
                           dim3(BLOCK), 0, c->stream, n, c->n_sys, w.off, w.grid, s7, d7,
                           w.xref[0], w.xref[1], w.xref[2], w.p4, w.summary);
    else
        hipLaunchKernelGGL(k_copy_disp, dim3(std::min(blocks_for(n), COPY_BLOCKS)), dim3(BLOCK),
                           0, c->stream, n, c->n_sys, w.off, w.grid, s7, d7, w.xref[0],
                           w.xref[1], w.xref[2], w.p4, w.summary);
}

lp_status rebuild_decision(lp_ctx* c, const double* const st[7], int force, bool first)
{
    Work& w = c->w;
    const int64_t n = c->n;
    // k_decide leaves the maximum at zero for the next captured step
    if (first) hipLaunchKernelGGL(k_disp_init, dim3(1), dim3(1), 0, c->stream, w.summary);
    c->disp_clear = false;
    // the state copied into the working state (in the current order) with
    // the displacement check; a rebuild then overwrites it
    if (n > 0) launch_copy_disp(c, st);
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(1), 0, c->stream, w.summary, w.gate,
                       w.cnt, force, w.bbox, c->n_sys);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "rebuild decision");
}

lp_status state_write_back(lp_ctx* c, double* const out[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (n > 0)
        for (int a = 0; a < 7; ++a)
            hipLaunchKernelGGL(k_copy_f64, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, n, w.sst[a], out[a], nullptr);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "state write-back");
}

lp_status list_check_start(lp_ctx* c, const double* const st[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    c->chk_pending = false;
    if (!c->list_ok) return LP_OK;
    // (a stencil build since the last check left the maximum at zero)
    if (!c->disp_clear)
        hipLaunchKernelGGL(k_disp_init, dim3(1), dim3(1), 0, c->stream, w.summary);
    c->disp_clear = false;
    if (n > 0) launch_copy_disp(c, st);
    hipError_t e = hipSuccess;
    if (!c->chk_ev) e = hipEventCreateWithFlags(&c->chk_ev, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w.h_summary, w.summary, sizeof(Summary), hipMemcpyDeviceToHost,
                           c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->chk_ev, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "displacement check");
    c->chk_pending = true;
    return LP_OK;
}

lp_status list_check_wait(lp_ctx* c, double* ratio)
{
    *ratio = -1.0;
    if (!c->chk_pending) return LP_OK;
    c->chk_pending = false;
    hipError_t e = hipEventSynchronize(c->chk_ev);
    if (e != hipSuccess) return hip_fail(c, e, "displacement check");
    const unsigned long long enc = c->w.h_summary->disp;
    const unsigned long long b = (enc >> 63) ? (enc & 0x7FFFFFFFFFFFFFFFull) : ~enc;
    double r;
    std::memcpy(&r, &b, sizeof(r));
    *ratio = r;
    return LP_OK;
}

}  // namespace lp
