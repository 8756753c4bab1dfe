// Neighbour search, stencil selection and ghost masks (Sec. 3.1 steps 5-6
// and the free-boundary ghosts of step 9).
//
// One thread per real particle scans the 27 cells around its own (real and
// mirror tables).  The exact stencil (nearest candidate of each octant,
// then the nearest others by key (r^2, id), m_max in all) is found without
// storing or sorting the candidate list:
//   pass A: count candidates, keep the nearest per octant, OR the octant
//           coverage bits, and histogram r^2 into 64 buckets of R^2/64
//           (byte counters in LDS);
//   the bucket holding the cut follows from the histogram;
//   pass B: rescan; emit octant-firsts and every candidate below the cut
//           bucket; candidates inside the cut bucket go to a per-thread
//           LDS list that is resolved exactly by key at the end.
// Bucketing is monotone in r^2, so the selected set equals the one a full
// sort by (r^2, id) gives.  Particles whose cut bucket overflows the list
// go to a slower path that collects and sorts all candidates.
#include "lp_internal.h"

namespace lp {

namespace {

inline unsigned int blocks_for(int64_t n, int per = BLOCK)
{
    return (unsigned int)((n + per - 1) / per);
}

struct Cand {
    double r2;
    int32_t id;
    int32_t oct;       // [dx>=0] + 2[dy>=0] + 4[dz>=0]
    int32_t cover;     // covered octant bit (0 if none)
};

__device__ __forceinline__ bool key_less(double ra, int32_t ia, double rb,
                                         int32_t ib)
{
    return ra < rb || (ra == rb && ia < ib);
}

// Visits every candidate of real i; f(Cand) is called in a fixed order.
template <class F>
__device__ __forceinline__ void for_candidates(const View& v, const GridInfo& g,
                                               int64_t i, double margin, F&& f)
{
    const double xi = v.x[i], yi = v.y[i], zi = v.z[i];
    int ix = (int)dmul(dsub(xi, g.x0), g.inv_c);
    int iy = (int)dmul(dsub(yi, g.y0), g.inv_c);
    int iz = (int)dmul(dsub(zi, g.z0), g.inv_c);
    ix = ix < 0 ? 0 : (ix >= g.nx ? g.nx - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= g.ny ? g.ny - 1 : iy);
    iz = iz < 0 ? 0 : (iz >= g.nz ? g.nz - 1 : iz);
    const double R2 = g.R2;
    auto test = [&](double xj, double yj, double zj, int32_t id) {
        const double dx = dsub(xj, xi), dy = dsub(yj, yi), dz = dsub(zj, zi);
        const double r2 = dist2(dx, dy, dz);
        if (r2 < R2 && id != (int32_t)i) {
            Cand c;
            c.r2 = r2;
            c.id = id;
            c.oct = (dx >= 0.0 ? 1 : 0) + (dy >= 0.0 ? 2 : 0) + (dz >= 0.0 ? 4 : 0);
            const bool far = fabs(dx) > margin && fabs(dy) > margin && fabs(dz) > margin;
            c.cover = far ? (1 << ((dx > 0.0 ? 1 : 0) + (dy > 0.0 ? 2 : 0) +
                                   (dz > 0.0 ? 4 : 0)))
                          : 0;
            f(c);
        }
    };
    for (int z = iz - 1; z <= iz + 1; ++z) {
        if (z < 0 || z >= g.nz) continue;
        for (int y = iy - 1; y <= iy + 1; ++y) {
            if (y < 0 || y >= g.ny) continue;
            const int64_t row = g.cell_base + (int64_t)g.nx * (y + (int64_t)g.ny * z);
            const int x0 = ix > 0 ? ix - 1 : 0;
            const int x1 = ix + 1 < g.nx ? ix + 1 : g.nx - 1;
            // the cells of a row are contiguous in the tables; real
            // particles of consecutive cells of a row are not (Z order),
            // so each cell is visited separately
            for (int x = x0; x <= x1; ++x) {
                const int64_t c = row + x;
                const int32_t a = v.cs[c], b = v.ce[c];
                for (int32_t j = a; j < b; ++j) test(v.x[j], v.y[j], v.z[j], j);
                const int32_t ma = v.mcs[c], mb = v.mce[c];
                for (int32_t q = ma; q < mb; ++q)
                    test(v.msx[q], v.msy[q], v.msz[q], v.msid[q]);
            }
        }
    }
}

__device__ __forceinline__ int bucket_of(double r2, double scale)
{
    const int b = (int)dmul(r2, scale);
    return b > HIST_BUCKETS - 1 ? HIST_BUCKETS - 1 : b;
}

__global__ __launch_bounds__(BLOCK) void k_stencil(View v, int32_t* hard,
                                                   unsigned int* hard_n,
                                                   int force_sorted)
{
    __shared__ uint32_t hist[HIST_BUCKETS / 4][BLOCK];
    __shared__ double lr2[LIST_CAP][BLOCK];
    __shared__ int32_t lid[LIST_CAP][BLOCK];
    const int t = threadIdx.x;
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + t;
    if (i >= v.n) return;
    const int s = sys_of(v.off, v.n_sys, i);
    const GridInfo& g = v.grid[s];
    const double margin = dmul(v.ghost_margin, g.h);
    const double scale = (double)HIST_BUCKETS / g.R2;
    for (int q = 0; q < HIST_BUCKETS / 4; ++q) hist[q][t] = 0u;

    // ---- pass A
    int nc = 0, covered = 0;
    double br2[8];
    int32_t bid[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        br2[o] = INFINITY;
        bid[o] = 0x7FFFFFFF;
    }
    for_candidates(v, g, i, margin, [&](const Cand& c) {
        ++nc;
        covered |= c.cover;
        double cr = br2[0];
        int32_t ci = bid[0];
#pragma unroll
        for (int o = 1; o < 8; ++o)
            if (c.oct == o) {
                cr = br2[o];
                ci = bid[o];
            }
        if (key_less(c.r2, c.id, cr, ci)) {
#pragma unroll
            for (int o = 0; o < 8; ++o)
                if (c.oct == o) {
                    br2[o] = c.r2;
                    bid[o] = c.id;
                }
        }
        const int b = bucket_of(c.r2, scale);
        hist[b >> 2][t] += 1u << (8 * (b & 3));
    });
    const int m_max = v.m_max;
    v.gmask[i] = (uint8_t)(~covered & 0xFF);
    const bool keep_all = nc <= m_max;
    int bstar = HIST_BUCKETS, need = 0;
    bool partial = false;
    if (!keep_all) {
        int n_oct = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o)
            if (bid[o] != 0x7FFFFFFF) {
                ++n_oct;
                const int b = bucket_of(br2[o], scale);
                hist[b >> 2][t] -= 1u << (8 * (b & 3));
            }
        const int K = m_max - n_oct;
        if (K < 0 || nc > 255) {
            // more octant-firsts than the cap, or byte counters could wrap
            v.scnt[i] = -1;
            const unsigned int slot = atomicAdd(hard_n, 1u);
            hard[slot] = (int32_t)i;
            return;
        }
        int cum = 0, hc = 0;
        for (int b = 0; b < HIST_BUCKETS; ++b) {
            hc = (int)((hist[b >> 2][t] >> (8 * (b & 3))) & 255u);
            if (cum + hc >= K) {
                bstar = b;
                need = K - cum;
                break;
            }
            cum += hc;
        }
        partial = need < hc;
        if (force_sorted || (partial && hc > LIST_CAP)) {
            v.scnt[i] = -1;
            const unsigned int slot = atomicAdd(hard_n, 1u);
            hard[slot] = (int32_t)i;
            return;
        }
    } else if (force_sorted) {
        v.scnt[i] = -1;
        const unsigned int slot = atomicAdd(hard_n, 1u);
        hard[slot] = (int32_t)i;
        return;
    }

    // ---- pass B
    int k = 0, nl = 0;
    const int64_t n = v.n;
    int32_t* sten = v.sten;
    for_candidates(v, g, i, margin, [&](const Cand& c) {
        bool emit;
        if (keep_all) {
            emit = true;
        } else {
            int32_t first = bid[0];
#pragma unroll
            for (int o = 1; o < 8; ++o)
                if (c.oct == o) first = bid[o];
            const int b = bucket_of(c.r2, scale);
            if (c.id == first || b < bstar) {
                emit = true;
            } else if (b == bstar) {
                if (partial) {
                    if (nl < LIST_CAP) {
                        lr2[nl][t] = c.r2;
                        lid[nl][t] = c.id;
                        ++nl;
                    }
                    emit = false;
                } else {
                    emit = true;
                }
            } else {
                emit = false;
            }
        }
        if (emit && k < m_max) {
            sten[(int64_t)k * n + i] = c.id;
            ++k;
        }
    });
    if (partial) {
        // the `need` smallest keys of the cut bucket
        for (int a = 0; a < nl; ++a) {
            int rank = 0;
            for (int b = 0; b < nl; ++b)
                if (key_less(lr2[b][t], lid[b][t], lr2[a][t], lid[a][t])) ++rank;
            if (rank < need && k < m_max) {
                sten[(int64_t)k * n + i] = lid[a][t];
                ++k;
            }
        }
    }
    v.scnt[i] = k;
}

// Exact path: collect all candidates, sort by key, take octant-firsts then
// the nearest others (the stencil rule written out directly).
__global__ __launch_bounds__(BLOCK) void k_stencil_sorted(
    View v, const int32_t* hard, const unsigned int* hard_n, double* sr2,
    int32_t* sid, ErrWord* err, Counters* cnt)
{
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    const unsigned int total = *hard_n;
    if (slot == 0) atomicAdd(&cnt->hard_stencils, (unsigned long long)total);
    double* r2s = sr2 + slot * HARD_CAP;
    int32_t* ids = sid + slot * HARD_CAP;
    for (int64_t tt = slot; tt < (int64_t)total; tt += nthreads) {
        const int64_t i = hard[tt];
        const int s = sys_of(v.off, v.n_sys, i);
        const GridInfo& g = v.grid[s];
        const double margin = dmul(v.ghost_margin, g.h);
        int nc = 0, covered = 0;
        for_candidates(v, g, i, margin, [&](const Cand& c) {
            covered |= c.cover;
            if (nc < HARD_CAP) {
                // insertion by key (ascending)
                int p = nc;
                while (p > 0 && key_less(c.r2, c.id, r2s[p - 1], ids[p - 1] & 0x0FFFFFFF)) {
                    r2s[p] = r2s[p - 1];
                    ids[p] = ids[p - 1];
                    --p;
                }
                r2s[p] = c.r2;
                ids[p] = c.id | (c.oct << 28);
            }
            ++nc;
        });
        v.gmask[i] = (uint8_t)(~covered & 0xFF);
        if (nc > HARD_CAP) {
            raise_error(err, ERR_CAPACITY, i);
            v.scnt[i] = 0;
            continue;
        }
        int firstpos[8];
        for (int o = 0; o < 8; ++o) firstpos[o] = -1;
        for (int p = 0; p < nc; ++p) {
            const int o = (ids[p] >> 28) & 7;
            if (firstpos[o] < 0) firstpos[o] = p;
        }
        int k = 0;
        const int m_max = v.m_max;
        for (int o = 0; o < 8; ++o)
            if (firstpos[o] >= 0 && k < m_max)
                v.sten[(int64_t)k++ * v.n + i] = ids[firstpos[o]] & 0x0FFFFFFF;
        for (int p = 0; p < nc && k < m_max; ++p) {
            bool f = false;
            for (int o = 0; o < 8; ++o) f = f || (firstpos[o] == p);
            if (!f) v.sten[(int64_t)k++ * v.n + i] = ids[p] & 0x0FFFFFFF;
        }
        v.scnt[i] = k;
    }
}

// ---- exports -----------------------------------------------------------

__global__ void k_count_candidates(View v, int64_t* counts /* n+1, at 1.. */)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) counts[0] = 0;
    if (i >= v.n) return;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    int nc = 0;
    for_candidates(v, g, i, 0.0, [&](const Cand&) { ++nc; });
    counts[i + 1] = nc;
}

// inclusive scan in place (single block of 1024) of counts[1..n]
__global__ void k_scan_i64(int64_t* a, int64_t n)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t b = 1 + t * chunk;
    const int64_t e = (b + chunk < n + 1) ? b + chunk : n + 1;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += a[i];
    part[t] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - s;
    for (int64_t i = b; i < e; ++i) {
        run += a[i];
        a[i] = run;
    }
}

__global__ void k_write_candidates(View v, const int64_t* off, int32_t* idx)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    int32_t* out = idx + off[i];
    int nc = 0;
    for_candidates(v, g, i, 0.0, [&](const Cand& c) {
        int p = nc++;
        while (p > 0 && out[p - 1] > c.id) {
            out[p] = out[p - 1];
            --p;
        }
        out[p] = c.id;
    });
}

__global__ void k_export_stencils(View v, int32_t* cnt_out, int32_t* idx_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    const int mm = v.m_max;
    const int m = min(max(v.scnt[i], 0), mm);
    if (cnt_out) cnt_out[i] = v.scnt[i];
    if (!idx_out) return;
    int32_t* out = idx_out + i * mm;
    for (int k = 0; k < m; ++k) {
        const int32_t id = v.sten[(int64_t)k * v.n + i];
        int p = k;
        while (p > 0 && out[p - 1] > id) {
            out[p] = out[p - 1];
            --p;
        }
        out[p] = id;
    }
    for (int k = m; k < mm; ++k) out[k] = -1;
}

__global__ void k_copy_u8(int64_t n, const uint8_t* a, uint8_t* b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

}  // namespace

lp_status stencils_build(lp_ctx* c, const double* const st[7])
{
    Work& w = c->w;
    const int64_t n = c->n;
    c->stencils_ok = false;
    if (!c->cells_ok) {
        c->err = "lp_build_cells must precede the stencil build";
        return LP_E_STATE;
    }
    View v = make_view(c, st);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, c->stream, w.hard_n);
    if (n > 0) {
        const int force = (c->cfg.debug_flags & LP_DEBUG_SORTED_STENCIL) ? 1 : 0;
        prof_mark(c, 1, false);
        hipLaunchKernelGGL(k_stencil, dim3(blocks_for(n)), dim3(BLOCK), 0,
                           c->stream, v, w.hard, w.hard_n, force);
        prof_mark(c, 1, true);
        prof_mark(c, 2, false);
        hipLaunchKernelGGL(k_stencil_sorted, dim3(HARD_SLOTS / BLOCK), dim3(BLOCK),
                           0, c->stream, v, w.hard, w.hard_n, w.hard_r2, w.hard_id,
                           w.err, w.cnt);
        prof_mark(c, 2, true);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "stencil launch");
    c->stencils_ok = true;
    return LP_OK;
}

lp_status stencils_export(lp_ctx* c, const double* const st[7],
                          int64_t* cand_off, int32_t* cand_idx, int64_t cap,
                          int64_t* needed, int32_t* sten_cnt,
                          int32_t* sten_idx, uint8_t* ghost_mask)
{
    Work& w = c->w;
    const int64_t n = c->n;
    View v = make_view(c, st);
    hipStream_t s = c->stream;
    if (cand_off || cand_idx || needed) {
        int64_t* off = cand_off ? cand_off : w.coff;
        hipLaunchKernelGGL(k_count_candidates, dim3(blocks_for(n + 1)), dim3(BLOCK),
                           0, s, v, off);
        hipLaunchKernelGGL(k_scan_i64, dim3(1), dim3(1024), 0, s, off, n);
        int64_t total = 0;
        hipError_t e = hipMemcpyAsync(&total, off + n, sizeof(int64_t),
                                      hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(c, e, "candidate count");
        if (needed) *needed = total;
        if (cand_idx) {
            if (total > cap) {
                c->err = "candidate capacity " + std::to_string(cap) +
                         " < needed " + std::to_string(total);
                return LP_E_CAPACITY;
            }
            if (n > 0)
                hipLaunchKernelGGL(k_write_candidates, dim3(blocks_for(n)),
                                   dim3(BLOCK), 0, s, v, off, cand_idx);
        }
    }
    if ((sten_cnt || sten_idx) && n > 0)
        hipLaunchKernelGGL(k_export_stencils, dim3(blocks_for(n)), dim3(BLOCK), 0,
                           s, v, sten_cnt, sten_idx);
    if (ghost_mask && n > 0)
        hipLaunchKernelGGL(k_copy_u8, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n,
                           w.gmask, ghost_mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "export launch");
    return LP_OK;
}

}  // namespace lp
