// Morton-sorted cell list and mirror particles (the paper's octree of
// Sec. 3.1 step 4 / Sec. 3.2 replaced by a uniform cell list sorted in
// Z order; mirrors of Sec. 3.1 step 9).
#include "lp_internal.h"

namespace lp {

namespace {

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

__global__ void k_bbox_init(unsigned long long* bbox, int n_sys,
                            unsigned long long* mcount)
{
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 6 * n_sys) bbox[t] = (t % 6) < 3 ? ~0ull : 0ull;
    if (t == 0) *mcount = 0;
}

constexpr int BBOX_CHUNK = 32;

__device__ void bbox_flush(unsigned long long* bbox, int s, const double* lo,
                           const double* hi)
{
    for (int a = 0; a < 3; ++a) {
        atomicMin(&bbox[6 * s + a], ord_enc(lo[a]));
        atomicMax(&bbox[6 * s + 3 + a], ord_enc(hi[a]));
    }
}

// Per-system bounding box of the real particles and the number of
// particles closer than R to their wall (the mirror count).
__global__ void k_bbox(int64_t n, int n_sys, const int64_t* off,
                       const lp_params* prm, const double* x,
                       const double* y, const double* z,
                       unsigned long long* bbox, unsigned long long* mcount)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t b = t * BBOX_CHUNK;
    const int lane = threadIdx.x & 63;
    int cur = -1;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    unsigned int mc = 0;
    if (b < n) {
        const int64_t e = (b + BBOX_CHUNK < n) ? b + BBOX_CHUNK : n;
        for (int64_t i = b; i < e; ++i) {
            int s = cur;
            if (s < 0 || i >= off[s + 1]) s = sys_of(off, n_sys, i);
            if (s != cur) {
                if (cur >= 0) bbox_flush(bbox, cur, lo, hi);
                cur = s;
                lo[0] = hi[0] = x[i];
                lo[1] = hi[1] = y[i];
                lo[2] = hi[2] = z[i];
            }
            double q[3] = {x[i], y[i], z[i]};
            for (int a = 0; a < 3; ++a) {
                lo[a] = fmin(lo[a], q[a]);
                hi[a] = fmax(hi[a], q[a]);
            }
            const lp_params& p = prm[s];
            if (dsub(z[i], p.wall_z) < p.R) ++mc;
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
    for (int off2 = 32; off2 > 0; off2 >>= 1) mc += __shfl_xor(mc, off2);
    if (lane == 0 && mc) atomicAdd(mcount, (unsigned long long)mc);
}

// Grid of each system from its bounding box; totals for the host.
__global__ void k_grid(int n_sys, const int64_t* off, const lp_params* prm,
                       const unsigned long long* bbox,
                       const unsigned long long* mcount, GridInfo* grid,
                       Summary* sum)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
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
        const double c = dmul(p.R, 1.0 + 1.0 / 1048576.0);
        g.inv_c = 1.0 / c;
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
            const double zm = dsub(dmul(2.0, p.wall_z), lo[2]);
            const double zt = zm > hi[2] ? zm : hi[2];
            const double ex = dmul(dsub(hi[0], g.x0), g.inv_c);
            const double ey = dmul(dsub(hi[1], g.y0), g.inv_c);
            const double ez = dmul(dsub(zt, g.z0), g.inv_c);
            if (!(ex < 65535.0 && ey < 65535.0 && ez < 65535.0)) {
                bad = 1;
                g.nx = g.ny = g.nz = 1;
            } else {
                g.nx = (int)ex + 1;
                g.ny = (int)ey + 1;
                g.nz = (int)ez + 1;
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
    sum->total_cells = base;
    sum->n_mirror = (int64_t)*mcount;
    sum->axis_bits = bits;
    sum->bad = bad;
}

__device__ __forceinline__ void cell_of(const GridInfo& g, double x, double y,
                                        double z, int& cx, int& cy, int& cz)
{
    int ix = (int)dmul(dsub(x, g.x0), g.inv_c);
    int iy = (int)dmul(dsub(y, g.y0), g.inv_c);
    int iz = (int)dmul(dsub(z, g.z0), g.inv_c);
    cx = ix < 0 ? 0 : (ix >= g.nx ? g.nx - 1 : ix);
    cy = iy < 0 ? 0 : (iy >= g.ny ? g.ny - 1 : iy);
    cz = iz < 0 ? 0 : (iz >= g.nz ? g.nz - 1 : iz);
}

// Sort keys (system, Morton code of the cell) and identity values.
__global__ void k_keys(int64_t n, int n_sys, const int64_t* off,
                       const GridInfo* grid, const double* x, const double* y,
                       const double* z, const int32_t* sys_src, int shift_sys,
                       unsigned long long* keys, int32_t* vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s = sys_src ? sys_of(off, n_sys, sys_src[i]) : sys_of(off, n_sys, i);
    const GridInfo& g = grid[s];
    int cx, cy, cz;
    cell_of(g, x[i], y[i], z[i], cx, cy, cz);
    keys[i] = ((unsigned long long)s << shift_sys) | morton3(cx, cy, cz);
    vals[i] = (int32_t)i;
}

// ---- stable LSD radix sort, 8-bit digits ------------------------------

__global__ void k_radix_hist(const unsigned long long* keys, int64_t n,
                             int shift, uint32_t* hist, int64_t nblk)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan in place of a uint32 array (single block of 1024).
__global__ void k_scan_u32(uint32_t* a, int64_t total)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (total + 1023) / 1024;
    const int64_t b = t * chunk;
    const int64_t e = (b + chunk < total) ? b + chunk : total;
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += a[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t i = b; i < e; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
}

__global__ void k_radix_scatter(const unsigned long long* kin,
                                const int32_t* vin, unsigned long long* kout,
                                int32_t* vout, int64_t n, int shift,
                                const uint32_t* hist, int64_t nblk)
{
    __shared__ uint32_t base[256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[BLOCK / 64][256];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    base[t] = hist[(int64_t)t * nblk + blockIdx.x];
    run[t] = 0;
    for (int w = 0; w < BLOCK / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const int64_t tb = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = tb + (int64_t)r * BLOCK + t;
        const bool valid = i < n;
        const unsigned long long key = valid ? kin[i] : 0ull;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        unsigned long long peers = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
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
        uint32_t add = 0;
        for (int w = 0; w < BLOCK / 64; ++w) {
            add += wcnt[w][t];
            wcnt[w][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

__global__ void k_gather7(int64_t n, const int32_t* perm,
                          const double* i0, const double* i1, const double* i2,
                          const double* i3, const double* i4, const double* i5,
                          const double* i6, double* o0, double* o1, double* o2,
                          double* o3, double* o4, double* o5, double* o6)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = perm[i];
    o0[i] = i0[j]; o1[i] = i1[j]; o2[i] = i2[j]; o3[i] = i3[j];
    o4[i] = i4[j]; o5[i] = i5[j]; o6[i] = i6[j];
}

__global__ void k_copy_i32(int64_t n, const int32_t* a, int32_t* b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_copy_f64(int64_t n, const double* a, double* b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_fill_i32(int64_t n, int32_t* a, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// ---- mirror compaction (exclusive scan of the wall flags) ------------

__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum,
                                                    uint32_t& total)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t inc = v;
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
        if (w < wave) pre += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    total = tot;
    return pre + inc - v;
}

__device__ __forceinline__ bool wall_flag(const int64_t* off, int n_sys,
                                          const GridInfo* grid, const double* z,
                                          int64_t i)
{
    const GridInfo& g = grid[sys_of(off, n_sys, i)];
    return dsub(z[i], g.wall) < g.R;
}

__global__ void k_mirror_count(int64_t n, int n_sys, const int64_t* off,
                               const GridInfo* grid, const double* z,
                               int32_t* bsum)
{
    __shared__ uint32_t wsum[BLOCK / 64];
    const int64_t b = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * SORT_ITEMS;
    uint32_t c = 0;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = b + r;
        if (i < n && wall_flag(off, n_sys, grid, z, i)) ++c;
    }
    uint32_t tot;
    block_excl_scan(c, wsum, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = (int32_t)tot;
}

__global__ void k_mirror_write(int64_t n, int n_sys, const int64_t* off,
                               const GridInfo* grid, const int32_t* bsum,
                               const double* x, const double* y,
                               const double* z, const double* u,
                               const double* v, const double* w,
                               const double* V, double* mx, double* my,
                               double* mz, double* mu, double* mv, double* mw,
                               double* mV, int32_t* msrc)
{
    __shared__ uint32_t wsum[BLOCK / 64];
    const int64_t b = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * SORT_ITEMS;
    uint32_t c = 0;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = b + r;
        if (i < n && wall_flag(off, n_sys, grid, z, i)) ++c;
    }
    uint32_t tot;
    uint32_t k = block_excl_scan(c, wsum, tot) + (uint32_t)bsum[blockIdx.x];
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = b + r;
        if (i < n && wall_flag(off, n_sys, grid, z, i)) {
            const GridInfo& g = grid[sys_of(off, n_sys, i)];
            mx[k] = x[i];
            my[k] = y[i];
            mz[k] = dsub(dmul(2.0, g.wall), z[i]);
            mu[k] = u[i];
            mv[k] = v[i];
            mw[k] = -w[i];
            mV[k] = V[i];
            msrc[k] = (int32_t)i;
            ++k;
        }
    }
}

__global__ void k_mirror_order(int64_t nm, int64_t n, const int32_t* order,
                               const double* mx, const double* my,
                               const double* mz, double* sx, double* sy,
                               double* sz, int32_t* sid)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nm) return;
    const int32_t k = order[q];
    sx[q] = mx[k];
    sy[q] = my[k];
    sz[q] = mz[k];
    sid[q] = (int32_t)(n + k);
}

// Cell start/end from sorted keys; positions give the linear cell index.
__global__ void k_cell_bounds(int64_t cnt, int n_sys, const int64_t* off,
                              const GridInfo* grid,
                              const unsigned long long* keys,
                              const double* x, const double* y,
                              const double* z, const int32_t* sys_src,
                              int32_t* cs, int32_t* ce)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const unsigned long long k = keys[i];
    const bool first = (i == 0) || keys[i - 1] != k;
    const bool last = (i == cnt - 1) || keys[i + 1] != k;
    if (!first && !last) return;
    const int s = sys_src ? sys_of(off, n_sys, sys_src[i]) : sys_of(off, n_sys, i);
    const GridInfo& g = grid[s];
    int cx, cy, cz;
    cell_of(g, x[i], y[i], z[i], cx, cy, cz);
    const int64_t c = g.cell_base + cx + (int64_t)g.nx * (cy + (int64_t)g.ny * cz);
    if (first) cs[c] = (int32_t)i;
    if (last) ce[c] = (int32_t)(i + 1);
}

__global__ void k_gather_src(int64_t nm, const int32_t* order,
                             const int32_t* msrc, int32_t* out)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < nm) out[q] = msrc[order[q]];
}

__global__ void k_set_i64(int64_t* p, int64_t v) { *p = v; }

inline unsigned int blocks_for(int64_t n, int per = BLOCK)
{
    return (unsigned int)((n + per - 1) / per);
}

// Sorts (keys, vals) of length cnt over `bits` bits; returns the buffers
// holding the result through kr / vr.
void radix_sort(lp_ctx* c, int64_t cnt, int bits, unsigned long long*& kr,
                int32_t*& vr)
{
    Work& w = c->w;
    unsigned long long* kin = w.keys0;
    unsigned long long* kout = w.keys1;
    int32_t* vin = w.vals0;
    int32_t* vout = w.vals1;
    const int64_t nblk = (cnt + SORT_TILE - 1) / SORT_TILE;
    const int passes = bits <= 0 ? 0 : (bits + 7) / 8;
    for (int p = 0; p < passes && cnt > 0; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(BLOCK), 0,
                           c->stream, kin, cnt, shift, w.hist, nblk);
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, c->stream,
                           w.hist, 256 * nblk);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(BLOCK),
                           0, c->stream, kin, vin, kout, vout, cnt, shift,
                           w.hist, nblk);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    kr = kin;
    vr = vin;
}

}  // namespace

lp_status cells_build(lp_ctx* c, double* const st[7], int32_t* perm_out,
                      bool write_back, double* const out[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    const int ns = c->n_sys;
    hipStream_t s = c->stream;
    c->cells_ok = false;
    c->stencils_ok = false;

    hipLaunchKernelGGL(k_bbox_init, dim3(blocks_for(6 * ns)), dim3(BLOCK), 0,
                       s, w.bbox, ns, w.mcount);
    if (n > 0)
        hipLaunchKernelGGL(k_bbox, dim3(blocks_for((n + BBOX_CHUNK - 1) / BBOX_CHUNK)),
                           dim3(BLOCK), 0, s, n, ns, w.off, w.prm, st[0], st[1],
                           st[2], w.bbox, w.mcount);
    hipLaunchKernelGGL(k_grid, dim3(1), dim3(64), 0, s, ns, w.off, w.prm,
                       w.bbox, w.mcount, w.grid, w.summary);
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
    c->axis_bits = sm.axis_bits;
    c->total_cells = sm.total_cells;
    c->n_mirror = sm.n_mirror;
    int sys_bits = 0;
    while ((1 << sys_bits) < ns) ++sys_bits;
    const int shift_sys = 3 * sm.axis_bits;
    const int bits = shift_sys + sys_bits;

    // sort the real particles
    unsigned long long* kr = nullptr;
    int32_t* vr = nullptr;
    if (n > 0) {
        hipLaunchKernelGGL(k_keys, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, ns,
                           w.off, w.grid, st[0], st[1], st[2],
                           (const int32_t*)nullptr, shift_sys, w.keys0, w.vals0);
        radix_sort(c, n, bits, kr, vr);
        hipLaunchKernelGGL(k_gather7, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n,
                           vr, st[0], st[1], st[2], st[3], st[4], st[5], st[6],
                           w.sst[0], w.sst[1], w.sst[2], w.sst[3], w.sst[4],
                           w.sst[5], w.sst[6]);
        if (perm_out)
            hipLaunchKernelGGL(k_copy_i32, dim3(blocks_for(n)), dim3(BLOCK), 0, s,
                               n, vr, perm_out);
    }
    const int64_t tc = sm.total_cells;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(tc)), dim3(BLOCK), 0, s, tc, w.cs, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(tc)), dim3(BLOCK), 0, s, tc, w.ce, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(tc)), dim3(BLOCK), 0, s, tc, w.mcs, 0);
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(tc)), dim3(BLOCK), 0, s, tc, w.mce, 0);
    if (n > 0)
        hipLaunchKernelGGL(k_cell_bounds, dim3(blocks_for(n)), dim3(BLOCK), 0, s,
                           n, ns, w.off, w.grid, kr, w.sst[0], w.sst[1], w.sst[2],
                           (const int32_t*)nullptr, w.cs, w.ce);

    // mirrors, in ascending order of their (sorted) source
    const int64_t nm = sm.n_mirror;
    if (n > 0) {
        const int64_t nb = (n + SORT_TILE - 1) / SORT_TILE;
        hipLaunchKernelGGL(k_mirror_count, dim3((unsigned)nb), dim3(BLOCK), 0, s,
                           n, ns, w.off, w.grid, w.sst[2], w.bsum);
        hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, s,
                           (uint32_t*)w.bsum, nb);
        hipLaunchKernelGGL(k_mirror_write, dim3((unsigned)nb), dim3(BLOCK), 0, s,
                           n, ns, w.off, w.grid, w.bsum, w.sst[0], w.sst[1],
                           w.sst[2], w.sst[3], w.sst[4], w.sst[5], w.sst[6],
                           w.mst[0], w.mst[1], w.mst[2], w.mst[3], w.mst[4],
                           w.mst[5], w.mst[6], w.msrc);
    }
    if (nm > 0) {
        hipLaunchKernelGGL(k_keys, dim3(blocks_for(nm)), dim3(BLOCK), 0, s, nm, ns,
                           w.off, w.grid, w.mst[0], w.mst[1], w.mst[2],
                           (const int32_t*)w.msrc, shift_sys, w.keys0, w.vals0);
        unsigned long long* mk = nullptr;
        int32_t* mv = nullptr;
        radix_sort(c, nm, bits, mk, mv);
        hipLaunchKernelGGL(k_mirror_order, dim3(blocks_for(nm)), dim3(BLOCK), 0, s,
                           nm, n, mv, w.mst[0], w.mst[1], w.mst[2], w.msx, w.msy,
                           w.msz, w.msid);
        // the system of cell-ordered mirror q is that of its source
        // msrc[order[q]]; the free value buffer holds those sources
        int32_t* srcs = (w.vals1 == mv) ? w.vals0 : w.vals1;
        hipLaunchKernelGGL(k_gather_src, dim3(blocks_for(nm)), dim3(BLOCK), 0, s,
                           nm, mv, w.msrc, srcs);
        hipLaunchKernelGGL(k_cell_bounds, dim3(blocks_for(nm)), dim3(BLOCK), 0, s,
                           nm, ns, w.off, w.grid, mk, w.msx, w.msy, w.msz,
                           (const int32_t*)srcs, w.mcs, w.mce);
    }
    hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(1), 0, s, w.n_mirror, nm);
    if (write_back && n > 0)
        for (int a = 0; a < 7; ++a)
            hipLaunchKernelGGL(k_copy_f64, dim3(blocks_for(n)), dim3(BLOCK), 0, s,
                               n, w.sst[a], out[a]);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "cell build launch");
    c->cells_ok = true;
    return LP_OK;
}

}  // namespace lp
