// Neighbour list, mirrors, stencil selection and ghost masks (Sec. 3.1
// steps 5-6 and the solid-wall mirrors and free-boundary ghosts of step 9).
//
// Neighbour list with skin: at a rebuild each particle records every real
// particle within R (1 + skin) and every potential mirror source (a real
// within R (1 + skin) of the wall whose reflection lies within R (1 + skin)).
// Until some particle has moved more than skin R / 2, the list contains
// every pair that can be closer than R, so every pass below applies the
// exact candidate test r2 = (dx*dx + dy*dy) + dz*dz < R*R to the list and
// obtains exactly the candidates a full search would.  The list is built
// with a wavefront per cell (k_list_cells: the cell's particles share the
// 27 cells they scan); k_list_build, a thread per particle, gives the same
// lists and serves as the check of the former.
//
// Stencil selection (nearest candidate of each octant, then the nearest
// others by key (r^2, id), m_max in all), one thread per particle, without
// storing or sorting the candidates:
//   pass 1: exact test of every list entry, count, octant coverage bits,
//           a histogram of r^2 in 64 buckets of R^2/64 (byte counters in
//           LDS) and the lowest bucket of each octant (which holds the
//           octant's first); each entry's bucket is stored as one byte;
//           the bucket holding the cut follows from the histogram;
//   pass 2: entries of lower buckets are kept (with them every octant
//           first below the cut); when the cut falls inside its bucket,
//           that bucket's few members are collected in a per-thread LDS
//           list, the firsts among them found and the rest ranked exactly
//           by key; an octant whose first lies above the cut (rare) gets
//           it from a scan of that one bucket.
// The result is a keep bitmask over the list entries (plus row count and
// ghost mask); the fits walk its set bits.  Bucketing is monotone in r^2,
// so the kept set equals the one a full sort by (r^2, id) gives.
// Particles whose cut bucket holds more members than the LDS list, or with
// more than 255 candidates, take a slower path that sorts all candidates.
#include "lp_visit.h"

#ifndef LP_SEL_BATCH
#define LP_SEL_BATCH 8
#endif

namespace lp {

namespace {

// List entries whose positions the selection gathers together.
constexpr int SEL_BATCH = LP_SEL_BATCH;
static_assert(SEL_BATCH % 4 == 0 && SEL_BATCH <= 8 && VCAP % SEL_BATCH == 0,
              "selection batches cover whole bucket-code words and one mask byte");

inline unsigned int blocks_for(int64_t n, int per = BLOCK)
{
    return (unsigned int)((n + per - 1) / per);
}

__device__ __forceinline__ void cell_clamp(const GridInfo& g, double x, double y,
                                           double z, int& cx, int& cy, int& cz)
{
    const double xw = wrap_coord(x, g.xlo, g.Lx), yw = wrap_coord(y, g.ylo, g.Ly);
    const int ix = (int)dmul(dsub(xw, g.x0), g.inv_cx);
    const int iy = (int)dmul(dsub(yw, g.y0), g.inv_cy);
    const int iz = (int)dmul(dsub(z, g.z0), g.inv_c);
    cx = ix < 0 ? 0 : (ix >= g.nx ? g.nx - 1 : ix);
    cy = iy < 0 ? 0 : (iy >= g.ny ? g.ny - 1 : iy);
    cz = iz < 0 ? 0 : (iz >= g.nz ? g.nz - 1 : iz);
}

// Orders the LDS accesses of one wavefront's lanes (no block barrier).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Neighbouring cell d in {-1, 0, 1} of cell c along an axis of nc cells:
// clipped on an open axis; wrapped on a periodic one, where fewer than
// three cells are each visited once.  -1: no cell.
__device__ __forceinline__ int nb_cell(int c, int d, int nc, bool periodic)
{
    if (!periodic) return (c + d < 0 || c + d >= nc) ? -1 : c + d;
    if (nc < 3 && (d == -1 || (nc == 1 && d == 1))) return -1;
    return (c + d + nc) % nc;
}

// ---- neighbour-list build ---------------------------------------------

// Candidates of the list build whose positions are loaded together.
constexpr int LIST_BATCH = 8;

// The candidates' positions come from their 32-byte records (x, y, z, 0),
// which the rebuild's gather writes: two loads per candidate.  Nearest
// images are taken only where some system is periodic (PERIODIC).
template <bool PERIODIC>
__global__ __launch_bounds__(BLOCK) void k_list_build(
    int64_t n, int n_sys, const int64_t* __restrict__ off,
    const GridInfo* __restrict__ grid, const double* __restrict__ x,
    const double* __restrict__ y, const double* __restrict__ z,
    const double* __restrict__ p4,
    const int32_t* __restrict__ cs, const int32_t* __restrict__ ce,
    int32_t* __restrict__ vl, int32_t* __restrict__ vcnt, ErrWord* err,
    const int32_t* gate)
{
    if (gate && *gate == 0) return;
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (i >= n) return;
    const GridInfo& g = grid[sys_of(off, n_sys, i)];
    const double Rv2 = g.Rv2 * (1.0 + 1e-12);
    const double xi = x[i], yi = y[i], zi = z[i];
    int cnt = 0;
    // entry cnt goes to out[cnt % VCHUNK]; out moves to the next chunk of
    // the particle (n VCHUNK entries on) whenever one fills
    int32_t* out = vl + (int64_t)i * VCHUNK;
    const int64_t cstride = n * VCHUNK;
    // the records as a byte base with 32-bit offsets (j < 2^27)
    const char* p4b = reinterpret_cast<const char*>(p4);
    const bool px = g.Lx > 0.0, py = g.Ly > 0.0;
    auto scan = [&](double qx, double qy, double qz, bool mirror) {
        int cx, cy, cz;
        cell_clamp(g, qx, qy, qz, cx, cy, cz);
        for (int zz = cz - 1; zz <= cz + 1; ++zz) {
            if (zz < 0 || zz >= g.nz) continue;
            for (int dy0 = -1; dy0 <= 1; ++dy0) {
                const int yy = nb_cell(cy, dy0, g.ny, py);
                if (yy < 0) continue;
                const int64_t row = g.cell_base + (int64_t)g.nx * (yy + (int64_t)g.ny * zz);
                // the particle ranges of the row's three cells, loaded
                // together (a clipped or repeated cell is empty)
                int32_t b[3], len[3];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const int xx = nb_cell(cx, q - 1, g.nx, px);
                    const int64_t c = row + (xx < 0 ? 0 : xx);
                    const int32_t cb = cs[c], cend = ce[c];
                    b[q] = cb;
                    len[q] = xx < 0 ? 0 : cend - cb;
                }
                const int l01 = len[0] + len[1];
                const int tot = l01 + len[2];
                // the row's candidates in cell order, LIST_BATCH at a time:
                // their positions loaded together, then tested in order
                for (int t0 = 0; t0 < tot; t0 += LIST_BATCH) {
                    int32_t jb[LIST_BATCH];
                    double qxs[LIST_BATCH], qys[LIST_BATCH], qzs[LIST_BATCH];
#pragma unroll
                    for (int u = 0; u < LIST_BATCH; ++u) {
                        const int t = t0 + u < tot ? t0 + u : t0;
                        const int32_t j = t < len[0] ? b[0] + t
                                          : (t < l01 ? b[1] + (t - len[0]) : b[2] + (t - l01));
                        jb[u] = j;
                        const double* r =
                            reinterpret_cast<const double*>(p4b + ((uint32_t)j << 5));
                        const double2 xy = *reinterpret_cast<const double2*>(r);
                        qxs[u] = xy.x;
                        qys[u] = xy.y;
                        qzs[u] = r[2];
                    }
#pragma unroll
                    for (int u = 0; u < LIST_BATCH; ++u) {
                        const int32_t j = jb[u];
                        if (t0 + u >= tot || (!mirror && j == (int32_t)i)) continue;
                        const double dx =
                            (PERIODIC ? image_coord(qxs[u], qx, g.Lx, g.hLx) : qxs[u]) - qx;
                        const double dy =
                            (PERIODIC ? image_coord(qys[u], qy, g.Ly, g.hLy) : qys[u]) - qy;
                        const double dz = qzs[u] - qz;
                        // the list only has to hold every pair within the
                        // list radius: fused products are fine here, their
                        // rounding far inside Rv2's 1e-12 margin
                        if (fma(dz, dz, fma(dy, dy, dx * dx)) >= Rv2) continue;
                        if (mirror && !(qzs[u] - g.wall < g.Rv)) continue;
                        if (cnt < VCAP) {
                            out[cnt & (VCHUNK - 1)] = mirror ? (j | MBIT) : j;
                            if ((cnt & (VCHUNK - 1)) == VCHUNK - 1) out += cstride;
                        }
                        ++cnt;
                    }
                }
            }
        }
    };
    scan(xi, yi, zi, false);
    // potential mirrors: reals near the wall whose reflection is near i,
    // i.e. reals near the reflection of i (reflection is an isometry)
    if (zi - g.wall < g.Rv) scan(xi, yi, dsub(dmul(2.0, g.wall), zi), true);
    if (cnt > VCAP) {
        raise_error(err, ERR_CAPACITY, i);
        cnt = VCAP;
    }
    vcnt[i] = cnt;
}

// ---- neighbour-list build, a wavefront per cell ------------------------
//
// Every particle of a cell scans the same 27 cells, so one wavefront takes
// a cell: the 27 cells' candidates, in the order the per-particle scan
// above visits them (rows by z, then y; a row's three cells by x; a cell's
// particles by index), form one sequence that is loaded 64 at a time, one
// candidate per lane, and tested against the cell's particles in turn.
// For each particle the accepted lanes append their ids in lane order (a
// ballot prefix count), so the lists are identical to the per-particle
// scan's (same entries, same order, same test on the same values).  A
// particle's potential mirror sources (the cells of its reflection, which
// differ between the particles of a cell) follow its real entries, one
// particle at a time, through the same sequence around the reflection.
// The cell's particles are taken 64 at a time; their positions sit in LDS
// (read with one address by the whole wavefront) and their running counts
// in lane q of `cntv`.
constexpr int LC_WAVES = BLOCK / 64;   // cells per block and pass
constexpr int LC_MAX_BLOCKS = 16384;   // grid-stride launches

__device__ __forceinline__ int sys_of_cell(const GridInfo* grid, int n_sys, int64_t c)
{
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (grid[mid].cell_base <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// entry pos of particle i, as vl_at places it; cst = n VCHUNK (< 2^30)
__device__ __forceinline__ void vl_put(int32_t* vl, int32_t i, uint32_t cst, uint32_t pos,
                                       int32_t e)
{
    vl[(uint64_t)(pos / VCHUNK) * cst + (uint64_t)(uint32_t)i * VCHUNK + pos % VCHUNK] = e;
}

// The 27 cells around (ccx, ccy, ccz) in scan order, cell l = 9 (z + 1) +
// 3 (y + 1) + (x + 1) for offsets x, y, z in {-1, 0, 1}: lane l < 27
// finds its cell's particle range (empty where the cell does not exist),
// and the wavefront stores the ranges' first particles and the exclusive
// prefix sums of their lengths (lanes 27..31: the total).  Returns the
// total.
__device__ __forceinline__ int cell_seq(const GridInfo& g, const int32_t* __restrict__ cs,
                                        const int32_t* __restrict__ ce, int ccx, int ccy,
                                        int ccz, int32_t* sb, int32_t* so)
{
    const int lane = threadIdx.x & 63;
    const bool px = g.Lx > 0.0, py = g.Ly > 0.0;
    int32_t b = 0, len = 0;
    if (lane < 27) {
        const int zz = ccz + lane / 9 - 1;
        const int yy = nb_cell(ccy, (lane / 3) % 3 - 1, g.ny, py);
        const int xx = nb_cell(ccx, lane % 3 - 1, g.nx, px);
        if (zz >= 0 && zz < g.nz && yy >= 0 && xx >= 0) {
            const int64_t c = g.cell_base + xx + (int64_t)g.nx * (yy + (int64_t)g.ny * zz);
            b = cs[c];
            len = ce[c] - b;
        }
    }
    int inc = len;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
    }
    if (lane < 32) {
        sb[lane] = b;
        so[lane] = inc - len;
    }
    wave_sync();
    return __builtin_amdgcn_readlane(inc, 31);
}

// Candidate t (< tot) of the sequence cell_seq stored: the last cell
// whose offset is at most t holds it (an empty cell shares its offset
// with the next one).  Lanes past the sequence take `dflt`.
__device__ __forceinline__ int32_t seq_at(const int32_t* sb, const int32_t* so, int t,
                                          int tot, int32_t dflt)
{
    int lo = 0, hi = 26;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const int mid = (lo + hi + 1) >> 1;
        if (so[mid] <= t) lo = mid; else hi = mid - 1;
    }
    return t < tot ? sb[lo] + (t - so[lo]) : dflt;
}

template <bool PERIODIC>
__global__ __launch_bounds__(BLOCK) void k_list_cells(
    int64_t n, int n_sys, const GridInfo* __restrict__ grid,
    const double* __restrict__ p4, const int32_t* __restrict__ cs,
    const int32_t* __restrict__ ce, int64_t n_cells, const int64_t* __restrict__ n_cells_dev,
    int32_t* __restrict__ vl, int32_t* __restrict__ vcnt, ErrWord* err,
    const int32_t* gate)
{
    if (gate && *gate == 0) return;
    __shared__ double4 ppos[LC_WAVES][64];
    __shared__ int32_t seqb[LC_WAVES][32], seqo[LC_WAVES][32];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int32_t* sb = seqb[wv];
    int32_t* so = seqo[wv];
    const int64_t tc = n_cells_dev ? *n_cells_dev : n_cells;
    const int64_t groups = (tc + LC_WAVES - 1) / LC_WAVES;
    const char* p4b = reinterpret_cast<const char*>(p4);
    const uint32_t cst = (uint32_t)(n * VCHUNK);
    auto load_pos = [&](int32_t j, double& qx, double& qy, double& qz) {
        const double* r = reinterpret_cast<const double*>(p4b + ((uint32_t)j << 5));
        const double2 xy = *reinterpret_cast<const double2*>(r);
        qx = xy.x;
        qy = xy.y;
        qz = r[2];
    };
    for (int64_t grp = xcd_block(blockIdx.x, gridDim.x); grp < groups; grp += gridDim.x) {
        const int64_t cell = grp * LC_WAVES + wv;
        if (cell >= tc) break;
        const int32_t cb = cs[cell], cend = ce[cell];
        if (cend <= cb) continue;
        const GridInfo& g = grid[sys_of_cell(grid, n_sys, cell)];
        const int loc = (int)(cell - g.cell_base);
        const int cx = loc % g.nx, cy = (loc / g.nx) % g.ny, cz = loc / (g.nx * g.ny);
        const double Rv2 = g.Rv2 * (1.0 + 1e-12);
        const int tot = cell_seq(g, cs, ce, cx, cy, cz, sb, so);
        for (int32_t q0 = cb; q0 < cend; q0 += 64) {
            const int nq = cend - q0 < 64 ? cend - q0 : 64;
            const int32_t mi = q0 + lane;          // this lane's particle
            if (lane < nq) {
                const double2* r = reinterpret_cast<const double2*>(p4b + ((uint32_t)mi << 5));
                const double2 a = r[0], c2 = r[1];
                ppos[wv][lane] = make_double4(a.x, a.y, c2.x, 0.0);
            }
            wave_sync();
            int cntv = 0;
            // real candidates
            for (int t0 = 0; t0 < tot; t0 += 64) {
                const bool in = t0 + lane < tot;
                const int32_t j = seq_at(sb, so, t0 + lane, tot, cb);
                double qx, qy, qz;
                load_pos(j, qx, qy, qz);
                for (int q = 0; q < nq; ++q) {
                    const double4 pq = ppos[wv][q];
                    const int32_t iq = q0 + q;
                    const double dx =
                        (PERIODIC ? image_coord(qx, pq.x, g.Lx, g.hLx) : qx) - pq.x;
                    const double dy =
                        (PERIODIC ? image_coord(qy, pq.y, g.Ly, g.hLy) : qy) - pq.y;
                    const double dz = qz - pq.z;
                    const bool acc =
                        in && j != iq && !(fma(dz, dz, fma(dy, dy, dx * dx)) >= Rv2);
                    const uint64_t m = __ballot(acc);
                    if (m) {
                        const int c0 = __builtin_amdgcn_readlane(cntv, q);
                        const uint32_t pos = (uint32_t)c0 + __builtin_amdgcn_mbcnt_hi(
                                                 (uint32_t)(m >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if (acc && pos < (uint32_t)VCAP) vl_put(vl, iq, cst, pos, j);
                        cntv = lane == q ? c0 + __popcll(m) : cntv;
                    }
                }
            }
            // potential mirrors of each particle near the wall: reals near
            // the wall that lie near its reflection
            bool reseq = false;
            for (int q = 0; q < nq; ++q) {
                const double4 pq = ppos[wv][q];
                if (!(pq.z - g.wall < g.Rv)) continue;
                const int32_t iq = q0 + q;
                const double zm = dsub(dmul(2.0, g.wall), pq.z);
                int mx, my, mz;
                cell_clamp(g, pq.x, pq.y, zm, mx, my, mz);
                wave_sync();
                const int mtot = cell_seq(g, cs, ce, mx, my, mz, sb, so);
                reseq = true;
                int c = __builtin_amdgcn_readlane(cntv, q);
                for (int t0 = 0; t0 < mtot; t0 += 64) {
                    const int32_t j = seq_at(sb, so, t0 + lane, mtot, cb);
                    double qx, qy, qz;
                    load_pos(j, qx, qy, qz);
                    const double dx =
                        (PERIODIC ? image_coord(qx, pq.x, g.Lx, g.hLx) : qx) - pq.x;
                    const double dy =
                        (PERIODIC ? image_coord(qy, pq.y, g.Ly, g.hLy) : qy) - pq.y;
                    const double dz = qz - zm;
                    const bool acc = t0 + lane < mtot &&
                                     !(fma(dz, dz, fma(dy, dy, dx * dx)) >= Rv2) &&
                                     qz - g.wall < g.Rv;
                    const uint64_t m = __ballot(acc);
                    const uint32_t pos = (uint32_t)c + __builtin_amdgcn_mbcnt_hi(
                                             (uint32_t)(m >> 32),
                                             __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (acc && pos < (uint32_t)VCAP) vl_put(vl, iq, cst, pos, j | MBIT);
                    c += __popcll(m);
                }
                cntv = lane == q ? c : cntv;
            }
            if (lane < nq) {
                if (cntv > VCAP) {
                    raise_error(err, ERR_CAPACITY, mi);
                    cntv = VCAP;
                }
                vcnt[mi] = cntv;
            }
            // the next chunk's positions (and the cell's own sequence, if
            // a mirror scan replaced it) overwrite the LDS words
            wave_sync();
            if (reseq && q0 + 64 < cend) cell_seq(g, cs, ce, cx, cy, cz, sb, so);
        }
        wave_sync();
    }
}

// ---- mirrors of the current state --------------------------------------

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

// Wall flags of the SORT_ITEMS chunks of 64 particles from wb on (chunk q:
// particles wb + 64 q + lane, false past n) as wave masks, bit l for
// particle wb + 64 q + l; all heights are loaded before any test.  s_tile:
// the system of the whole tile, or -1 when the tile spans several.
__device__ __forceinline__ void wall_masks(int64_t n, int n_sys, const int64_t* off,
                                           const GridInfo* grid, const double* z, int64_t wb,
                                           int s_tile, uint64_t (&m)[SORT_ITEMS])
{
    const int lane = threadIdx.x & 63;
    double zz[SORT_ITEMS];
#pragma unroll
    for (int q = 0; q < SORT_ITEMS; ++q) {
        const int64_t i = wb + 64 * q + lane;
        zz[q] = i < n ? z[i] : INFINITY;
    }
    if (s_tile >= 0) {
        const double wall = grid[s_tile].wall, R = grid[s_tile].R;
#pragma unroll
        for (int q = 0; q < SORT_ITEMS; ++q) m[q] = __ballot(dsub(zz[q], wall) < R);
    } else {
#pragma unroll
        for (int q = 0; q < SORT_ITEMS; ++q) {
            const int64_t i = wb + 64 * q + lane;
            bool f = false;
            if (i < n) {
                const GridInfo& g = grid[sys_of(off, n_sys, i)];
                f = dsub(zz[q], g.wall) < g.R;
            }
            m[q] = __ballot(f);
        }
    }
}

// The system holding every particle of tile `tile`, or -1.
__device__ __forceinline__ int tile_system(int64_t n, int n_sys, const int64_t* off,
                                           int64_t tile)
{
    const int64_t t0 = tile * SORT_TILE;
    const int64_t t1 = t0 + SORT_TILE - 1 < n ? t0 + SORT_TILE - 1 : n - 1;
    const int s0 = sys_of(off, n_sys, t0);
    return s0 == sys_of(off, n_sys, t1) ? s0 : -1;
}

// Mirrors are counted and numbered a tile of SORT_TILE particles per block:
// wave w takes the SORT_ITEMS chunks of 64 consecutive particles from
// t0 + 64 SORT_ITEMS w on, one particle per lane (coalesced loads of z),
// with the wall flags of a chunk as one ballot mask.
constexpr int MIRROR_WAVES = BLOCK / 64;
static_assert(SORT_TILE == MIRROR_WAVES * 64 * SORT_ITEMS, "a tile per block");

// Also clears the step's counters: the selection's list of particles for
// the sorted path, the fits' refit list and the displacement maximum of
// the next list check (read by the host before this kernel is enqueued).
__global__ void k_mirror_count(int64_t n, int n_sys, const int64_t* off,
                               const GridInfo* grid, const double* z,
                               int32_t* bsum, unsigned int* hard_n,
                               unsigned int* redo_n, Summary* sum)
{
    __shared__ uint32_t wsum[MIRROR_WAVES];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *hard_n = 0u;
        *redo_n = 0u;
        sum->disp = DISP_ZERO;
    }
    const int w = threadIdx.x >> 6;
    const int s_tile = tile_system(n, n_sys, off, blockIdx.x);
    const int64_t wb = (int64_t)blockIdx.x * SORT_TILE + (int64_t)w * 64 * SORT_ITEMS;
    uint64_t m[SORT_ITEMS];
    wall_masks(n, n_sys, off, grid, z, wb, s_tile, m);
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < SORT_ITEMS; ++q) c += (uint32_t)__popcll(m[q]);
    if ((threadIdx.x & 63) == 0) wsum[w] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
#pragma unroll
        for (int q = 0; q < MIRROR_WAVES; ++q) tot += wsum[q];
        bsum[blockIdx.x] = (int32_t)tot;
    }
}

// Exclusive scan in place of a uint32 array (single block of 1024); the
// total goes to *total.
__global__ void k_scan_total(uint32_t* a, int64_t cnt, int64_t* total)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (cnt + 1023) / 1024;
    const int64_t b = t * chunk;
    const int64_t e = (b + chunk < cnt) ? b + chunk : cnt;
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
    if (t == 1023) *total = (int64_t)part[1023];
}

// bsum holds the blocks' exclusive offsets (scanned) or their counts; with
// counts (few blocks) each block sums those of the blocks before it and the
// last block writes the total.  Mirror ids follow the source order.
__global__ void k_mirror_write(int64_t n, int n_sys, const int64_t* off,
                               const GridInfo* grid, const int32_t* bsum,
                               int scanned, int64_t* total, const double* z,
                               int32_t* mirror_of, int32_t* msrc)
{
    __shared__ uint32_t wsum[MIRROR_WAVES];
    __shared__ uint32_t bpre[MIRROR_WAVES];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t base;
    if (scanned) {
        base = (uint32_t)bsum[blockIdx.x];
    } else {
        uint32_t p = 0;
        for (int q = threadIdx.x; q < (int)blockIdx.x; q += BLOCK) p += (uint32_t)bsum[q];
        for (int d = 32; d > 0; d >>= 1) p += __shfl_xor(p, d);
        if (lane == 0) bpre[w] = p;
        __syncthreads();
        base = 0;
#pragma unroll
        for (int q = 0; q < MIRROR_WAVES; ++q) base += bpre[q];
    }
    const int s_tile = tile_system(n, n_sys, off, blockIdx.x);
    const int64_t wb = (int64_t)blockIdx.x * SORT_TILE + (int64_t)w * 64 * SORT_ITEMS;
    uint64_t m[SORT_ITEMS];
    wall_masks(n, n_sys, off, grid, z, wb, s_tile, m);
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < SORT_ITEMS; ++q) c += (uint32_t)__popcll(m[q]);
    if (lane == 0) wsum[w] = c;
    __syncthreads();
    uint32_t k = base, tot = 0;
#pragma unroll
    for (int q = 0; q < MIRROR_WAVES; ++q) {
        k += q < w ? wsum[q] : 0u;
        tot += wsum[q];
    }
    if (!scanned && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        *total = (int64_t)(base + tot);
    const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
    for (int q = 0; q < SORT_ITEMS; ++q) {
        const int64_t i = wb + 64 * q + lane;
        if (i < n) {
            const bool f = (m[q] >> lane) & 1ull;
            const uint32_t kk = k + (uint32_t)__popcll(m[q] & below);
            mirror_of[i] = f ? (int32_t)kk : -1;
            if (f) msrc[kk] = (int32_t)i;
        }
        k += (uint32_t)__popcll(m[q]);
    }
}

// ---- stencil selection ---------------------------------------------------

__device__ __forceinline__ int hist_get(const uint32_t (*hist)[BLOCK], int b, int t)
{
    return (int)((hist[b >> 2][t] >> (8 * (b & 3))) & 255u);
}

__device__ __forceinline__ void hist_add(uint32_t (*hist)[BLOCK], int b, int t,
                                         int d)
{
    hist[b >> 2][t] += (uint32_t)d << (8 * (b & 3));
}

// First bucket whose cumulative count reaches K; need = how many of its
// members are kept, hc = its count.
__device__ __forceinline__ int cut_bucket(const uint32_t (*hist)[BLOCK], int t,
                                          int K, int& need, int& hc)
{
    int cum = 0;
    for (int b = 0; b < HIST_BUCKETS; ++b) {
        hc = hist_get(hist, b, t);
        if (cum + hc >= K) {
            need = K - cum;
            return b;
        }
        cum += hc;
    }
    need = 0;
    hc = 0;
    return HIST_BUCKETS;
}

// keep mask over the list entries of one particle (VCAP bits)
struct Mask4 {
    uint64_t w0 = 0, w1 = 0, w2 = 0, w3 = 0;
    __device__ __forceinline__ void set(int k)
    {
        const uint64_t b = 1ull << (k & 63);
        if (k < 64)
            w0 |= b;
        else if (k < 128)
            w1 |= b;
        else if (k < 192)
            w2 |= b;
        else
            w3 |= b;
    }
    // bits of `bits` at entries k0, k0 + 1, ... (W bits, k0 a multiple
    // of W, W dividing 64)
    template <int W = 8>
    __device__ __forceinline__ void set_bits(int k0, uint32_t bits)
    {
        const uint64_t b = (uint64_t)(bits & ((1u << W) - 1u)) << (k0 & 63);
        if (k0 < 64)
            w0 |= b;
        else if (k0 < 128)
            w1 |= b;
        else if (k0 < 192)
            w2 |= b;
        else
            w3 |= b;
    }
    __device__ __forceinline__ bool has(int k) const
    {
        const uint64_t w = k < 64 ? w0 : (k < 128 ? w1 : (k < 192 ? w2 : w3));
        return (w >> (k & 63)) & 1ull;
    }
};

__device__ __forceinline__ void write_rec(const View& v, int64_t i, int m, int gm,
                                          int mode, const Mask4& mk)
{
    static_assert(MASK_WORDS == 4, "four keep-mask words");
    const int64_t n = v.n;
    int32_t* q = v.rec;
    q[REC_M * n + i] = m;
    q[REC_GM * n + i] = gm;
    q[REC_MODE * n + i] = mode;
    v.kmask[i] = mk.w0;
    v.kmask[n + i] = mk.w1;
    v.kmask[2 * n + i] = mk.w2;
    v.kmask[3 * n + i] = mk.w3;
}

// Calls f(pt, dx, dy, dz, r2) for every candidate of particle i.
template <class F>
__device__ __forceinline__ void for_candidates(const View& v, const GridInfo& g,
                                               int64_t i, F&& f)
{
    const int64_t n = v.n;
    const double xi = v.x[i], yi = v.y[i], zi = v.z[i];
    const double R2 = g.R2;
    const int cnt = v.vcnt[i];
    for (int k = 0; k < cnt; ++k) {
        const Pt p = list_point(v, g, v.vl[vl_at(n, i, k)], xi, yi);
        if (!p.valid) continue;
        const double dx = dsub(p.x, xi), dy = dsub(p.y, yi), dz = dsub(p.z, zi);
        const double r2 = dist2(dx, dy, dz);
        if (r2 < R2) f(p, dx, dy, dz, r2);
    }
}

// The points of the SEL_BATCH list entries k0, k0 + 1, ... of particle i
// for the exact candidate test: positions from the 32-byte records, a
// mirror's position reflected and its existence taken from its source's
// height (a mirror exists while the source lies within R of the wall, the
// rule that sets mirror_of); no ids.  Entries past cnt are read (every
// particle holds VCAP list slots, so every read is in bounds) but stand
// for i itself and are not candidates.  The record offset j * 32 stays below 2^32 (j < 2^27).
template <bool PERIODIC>
__device__ __forceinline__ void select_gather(const View& v, const Seen& s,
                                              const GridInfo& g, int64_t i, int k0,
                                              int cnt, Pt (&p)[SEL_BATCH])
{
    const int64_t n = v.n;
    int32_t e[SEL_BATCH];
    vl_load(v.vl, n, i, k0, e);
#pragma unroll
    for (int u = 0; u < SEL_BATCH; ++u) e[u] = k0 + u < cnt ? e[u] : (int32_t)i;
    const char* base = reinterpret_cast<const char*>(v.p4);
#pragma unroll
    for (int u = 0; u < SEL_BATCH; ++u) {
        const uint32_t off = (uint32_t)(e[u] & ~MBIT) << 5;
        const double* r = reinterpret_cast<const double*>(base + off);
        const double2 xy = *reinterpret_cast<const double2*>(r);
        p[u].x = xy.x;
        p[u].y = xy.y;
        p[u].z = r[2];
        p[u].mirror = (e[u] & MBIT) != 0;
    }
#pragma unroll
    for (int u = 0; u < SEL_BATCH; ++u) {
        const double zs = p[u].z;
        p[u].valid = !p[u].mirror || dsub(zs, g.wall) < g.R;
        p[u].z = p[u].mirror ? dsub(s.wall2, zs) : zs;
        if (PERIODIC) {
            p[u].x = image_coord(p[u].x, s.xi, s.Lx, s.hLx);
            p[u].y = image_coord(p[u].y, s.yi, s.Ly, s.hLy);
        }
    }
}

template <bool PERIODIC>
__global__ __launch_bounds__(BLOCK) void k_select(View v, int32_t* hard,
                                                  unsigned int* hard_n,
                                                  int force_sorted)
{
    __shared__ uint32_t hist[HIST_BUCKETS / 4][BLOCK];
    // cut-bucket members, one word each: r^2 rounded to float with its
    // low 8 bits replaced by the list index.  Rounding and truncation are
    // monotone, so a smaller word means a smaller r^2; equal truncated
    // keys take the exact keys again.  loct: their octants (bit 7: the
    // member is its octant's first).
    __shared__ uint32_t lkey[LIST_CAP][BLOCK];
    __shared__ uint8_t loct[LIST_CAP][BLOCK];
    const int t = threadIdx.x;
    const int64_t i = xcd_block(blockIdx.x, gridDim.x) * BLOCK + t;
    if (i >= v.n) return;
    const int64_t n = v.n;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    const double margin = dmul(v.ghost_margin, g.h);
    const double scale = (double)HIST_BUCKETS / g.R2;
    const double R2 = g.R2;
    uint32_t* __restrict__ code = v.code;
    const Seen s = seen_from(v, g, i);
    const double xi = s.xi, yi = s.yi, zi = s.zi;
    const int cnt = v.vcnt[i];
#pragma unroll
    for (int q = 0; q < HIST_BUCKETS / 4; ++q) hist[q][t] = 0u;

    // ---- pass 1: exact test of every list entry, SEL_BATCH entries at a
    // time (their list words, then their positions, all in flight
    // together); the buckets are stored four to a word (word k / 4 of all
    // lanes at once: coalesced).  Per octant only the lowest bucket is
    // tracked: it holds the octant's first.  Those minima are LDS words
    // of the thread's member column (unused until the keep pass), lowered
    // with no-return atomic minima.
    int nc = 0, covered = 0;
    Mask4 cm;                          // candidate entries
#pragma unroll
    for (int o = 0; o < 8; ++o) lkey[o][t] = 0xFFu;
    for (int k0 = 0; k0 < cnt; k0 += SEL_BATCH) {
        Pt pb[SEL_BATCH];
        select_gather<PERIODIC>(v, s, g, i, k0, cnt, pb);
        uint32_t cw[SEL_BATCH / 4];
#pragma unroll
        for (int w = 0; w < SEL_BATCH / 4; ++w) cw[w] = 0xFFFFFFFFu;
        // Every entry of the batch takes the same instructions, predicated
        // on being a candidate (no divergent branches): the histogram gets
        // a no-return LDS add of 0 or 1, the other updates are selects.
        uint32_t bm = 0;               // candidates among the batch
#pragma unroll
        for (int u = 0; u < SEL_BATCH; ++u) {
            const Pt& p = pb[u];
            const double dx = dsub(p.x, xi), dy = dsub(p.y, yi), dz = dsub(p.z, zi);
            const double d2 = dist2(dx, dy, dz);
            const bool c = k0 + u < cnt && p.valid && d2 < R2;
            nc += c ? 1 : 0;
            bm |= c ? 1u << u : 0u;
            // a candidate farther than margin (>= 0) from i on every axis
            // covers its octant (no zero component, so octant_of is exact)
            const int oct = octant_of(dx, dy, dz);
            const bool far = fabs(dx) > margin && fabs(dy) > margin && fabs(dz) > margin;
            covered |= (c && far) ? 1 << oct : 0;
            const int bi = bucket_of(d2, scale);
            const uint32_t b = (uint32_t)(bi < 0 ? 0 : bi);
            atomicMin(&lkey[oct][t], c ? b : 0xFFu);
            atomicAdd(&hist[b >> 2][t], (c ? 1u : 0u) << (8u * (b & 3u)));
            const uint32_t cs = 8u * (uint32_t)(u & 3);
            cw[u >> 2] = c ? (cw[u >> 2] & ~(0xFFu << cs)) | (b << cs) : cw[u >> 2];
        }
        cm.set_bits(k0, bm);
#pragma unroll
        for (int w = 0; w < SEL_BATCH / 4; ++w)
            if (k0 + 4 * w < cnt) code[(int64_t)((k0 >> 2) + w) * n + i] = cw[w];
    }
    const int gm = ~covered & 0xFF;
    const int m_max = v.m_max;
    if (force_sorted || nc > 255) {
        write_rec(v, i, 0, gm, MODE_SORTED, Mask4());
        hard[atomicAdd(hard_n, 1u)] = (int32_t)i;
        return;
    }
    if (nc <= m_max) {
        write_rec(v, i, nc, gm, MODE_ALL, cm);
        return;
    }
    uint32_t mbv[8];
#pragma unroll
    for (int o = 0; o < 8; ++o) mbv[o] = lkey[o][t];
    auto minb = [&](int o) -> uint32_t { return mbv[o]; };
    int n_oct = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o)
        if (minb(o) != 0xFFu) {
            ++n_oct;
            hist_add(hist, (int)minb(o), t, -1);
        }
    const int K = m_max - n_oct;
    int need = 0, hc = 0;
    const int bstar = K < 0 ? 0 : cut_bucket(hist, t, K, need, hc);
    // octants whose first lies in the cut bucket (B) or above it (C); the
    // others' firsts lie below the cut and are kept with their buckets
    uint32_t octB = 0, octC = 0;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        const uint32_t mo = minb(o);
        if (mo == (uint32_t)bstar) octB |= 1u << o;
        else if (mo != 0xFFu && mo > (uint32_t)bstar) octC |= 1u << o;
    }
    const int nB = __popc(octB);
    const bool partial = need < hc;
    if (K < 0 || (partial && hc + nB > LIST_CAP)) {
        write_rec(v, i, 0, gm, MODE_SORTED, Mask4());
        hard[atomicAdd(hard_n, 1u)] = (int32_t)i;
        return;
    }

    // ---- pass 2: keep every lower bucket; the cut bucket whole, or its
    // members collected for exact ranking
    // Sixteen entries at a time: their keep and member bits are formed
    // with selects (no divergent branch per entry); the few members are
    // then listed from their bits.
    Mask4 mk;
    int nl = 0;
    const uint32_t ub = (uint32_t)bstar;
    for (int k0 = 0; k0 < cnt; k0 += 16) {
        uint32_t cw[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
            cw[w] = k0 + 4 * w < cnt ? code[(int64_t)((k0 >> 2) + w) * n + i] : 0xFFFFFFFFu;
        uint32_t keep = 0, memb = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const uint32_t kc = (cw[u >> 2] >> (8 * (u & 3))) & 0xFFu;
            keep |= (kc < ub || (kc == ub && !partial)) ? 1u << u : 0u;
            memb |= (kc == ub && partial) ? 1u << u : 0u;
        }
        mk.set_bits<16>(k0, keep);
        while (memb) {
            lkey[nl][t] = (uint32_t)(k0 + __builtin_ctz(memb));
            ++nl;
            memb &= memb - 1;
        }
    }
    // keys of the members: r^2 rounded to float with its low 8 bits
    // replaced by the list index, and their octants
    for (int a0 = 0; a0 < nl; a0 += 4) {
        int32_t e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            e[u] = a0 + u < nl ? v.vl[vl_at(n, i, lkey[a0 + u][t])] : (int32_t)i;
        Pt pb[4];
        gather_list(v, s, e, pb);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (a0 + u >= nl) continue;
            const Pt& p = pb[u];
            const double dx = dsub(p.x, xi), dy = dsub(p.y, yi), dz = dsub(p.z, zi);
            const float f = (float)dist2(dx, dy, dz);
            lkey[a0 + u][t] = (__float_as_uint(f) & ~0xFFu) | lkey[a0 + u][t];
            loct[a0 + u][t] = (uint8_t)octant_of(dx, dy, dz);
        }
    }
    auto exact_key = [&](int k, double& r2, int32_t& id) {
        const int32_t e[1] = {v.vl[vl_at(n, i, k)]};
        Pt p[1];
        gather_list(v, s, e, p);
        r2 = dist2(dsub(p[0].x, xi), dsub(p[0].y, yi), dsub(p[0].z, zi));
        id = p[0].id;
    };
    // is member b's key (r^2, id) below member a's?
    auto below = [&](int b, int a) {
        const uint32_t ka = lkey[a][t], kb = lkey[b][t];
        if ((kb >> 8) != (ka >> 8)) return (kb >> 8) < (ka >> 8);
        double ra, rb;
        int32_t ia, ib;
        exact_key((int)(ka & 0xFFu), ra, ia);
        exact_key((int)(kb & 0xFFu), rb, ib);
        return key_less(rb, ib, ra, ia);
    };
    if (partial) {
        // firsts of the B octants among the members: kept, not ranked
        if (octB) {
            for (int a = 0; a < nl; ++a) {
                const int o = loct[a][t];
                if (!((octB >> o) & 1u)) continue;
                bool first = true;
                for (int b = 0; b < nl && first; ++b)
                    if (b != a && (loct[b][t] & 7) == o && below(b, a)) first = false;
                if (first) {
                    loct[a][t] = (uint8_t)(o | 0x80);
                    mk.set((int)(lkey[a][t] & 0xFFu));
                }
            }
        }
        // the `need` smallest keys of the other members
        for (int a = 0; a < nl; ++a) {
            if (loct[a][t] & 0x80) continue;
            int rank = 0;
            for (int b = 0; b < nl; ++b)
                if (b != a && !(loct[b][t] & 0x80) && below(b, a)) ++rank;
            if (rank < need) mk.set((int)(lkey[a][t] & 0xFFu));
        }
    }
    // firsts of the C octants (rare): the smallest key of the octant in
    // its lowest bucket
    if (octC) {
        for (int o = 0; o < 8; ++o) {
            if (!((octC >> o) & 1u)) continue;
            const int mo = (int)minb(o);
            double br = INFINITY;
            int32_t bi = NOID;
            int bk = -1;
            for (int k = 0; k < cnt; ++k) {
                if ((int)((code[(int64_t)(k >> 2) * n + i] >> (8 * (k & 3))) & 0xFFu) != mo)
                    continue;
                const Pt p = list_point(v, g, v.vl[vl_at(n, i, k)], xi, yi);
                const double dx = dsub(p.x, xi), dy = dsub(p.y, yi), dz = dsub(p.z, zi);
                if (octant_of(dx, dy, dz) != o) continue;
                const double r2 = dist2(dx, dy, dz);
                if (key_less(r2, p.id, br, bi)) {
                    br = r2;
                    bi = p.id;
                    bk = k;
                }
            }
            if (bk >= 0) mk.set(bk);
        }
    }
    write_rec(v, i, m_max, gm, 0, mk);
}

// Exact path, one wavefront per particle: the candidates are collected
// into LDS, each is ranked by key (r^2, id) against all others, and the
// stencil rule is applied directly (octant-firsts in octant order, then
// the others in key order, m_max in all).
__global__ __launch_bounds__(BLOCK) void k_select_sorted(
    View v, const int32_t* hard, const unsigned int* hard_n, ErrWord* err,
    Counters* cnt)
{
    constexpr int WPB = BLOCK / 64;
    constexpr int PER_LANE = HARD_CAP / 64;
    __shared__ double sr2[WPB][HARD_CAP];
    __shared__ int32_t sid[WPB][HARD_CAP];   // id | octant << 28
    __shared__ double fr2[WPB][8];
    __shared__ int32_t fid[WPB][8];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const unsigned int total = *hard_n;
    if (blockIdx.x == 0 && threadIdx.x == 0)
        atomicAdd(&cnt->hard_stencils, (unsigned long long)total);
    const int64_t n = v.n;
    const int m_max = v.m_max;
    const uint64_t below = (1ull << lane) - 1;
    for (int64_t tt = (int64_t)blockIdx.x * WPB + wv; tt < (int64_t)total;
         tt += (int64_t)gridDim.x * WPB) {
        const int64_t i = hard[tt];
        const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
        const double xi = v.x[i], yi = v.y[i], zi = v.z[i];
        const double R2 = g.R2;
        const int cnt_i = v.vcnt[i];
        // ---- collect (ballot compaction, list order)
        int nc = 0;
        for (int k0 = 0; k0 < cnt_i; k0 += 64) {
            const int k = k0 + lane;
            bool cand = false;
            double r2 = 0.0;
            int32_t key = 0;
            if (k < cnt_i) {
                const Pt p = list_point(v, g, v.vl[vl_at(n, i, k)], xi, yi);
                if (p.valid) {
                    const double dx = dsub(p.x, xi), dy = dsub(p.y, yi),
                                 dz = dsub(p.z, zi);
                    r2 = dist2(dx, dy, dz);
                    cand = r2 < R2;
                    key = p.id | (octant_of(dx, dy, dz) << 28);
                }
            }
            const uint64_t bal = __ballot(cand);
            const int pos = nc + __popcll(bal & below);
            if (cand && pos < HARD_CAP) {
                sr2[wv][pos] = r2;
                sid[wv][pos] = key;
            }
            nc += __popcll(bal);
        }
        if (nc > HARD_CAP) {
            if (lane == 0) {
                raise_error(err, ERR_CAPACITY, i);
                v.rec[REC_M * n + i] = 0;
            }
            continue;
        }
        if (lane < 8) {
            fr2[wv][lane] = INFINITY;
            fid[wv][lane] = -1;
        }
        wave_sync();
        // ---- rank of each candidate, overall and within its octant
        int rk[PER_LANE], ork[PER_LANE];
#pragma unroll
        for (int q = 0; q < PER_LANE; ++q) {
            const int c = lane + 64 * q;
            rk[q] = 0;
            ork[q] = 1;
            if (c < nc) {
                const double rc = sr2[wv][c];
                const int32_t kc = sid[wv][c];
                const int32_t idc = kc & 0x0FFFFFFF;
                const int oc = (kc >> 28) & 7;
                int r = 0, o = 0;
                for (int j = 0; j < nc; ++j) {
                    const int32_t kj = sid[wv][j];
                    const bool less = key_less(sr2[wv][j], kj & 0x0FFFFFFF, rc, idc);
                    r += less ? 1 : 0;
                    o += (less && ((kj >> 28) & 7) == oc) ? 1 : 0;
                }
                rk[q] = r;
                ork[q] = o;
                if (o == 0) {
                    fr2[wv][oc] = rc;
                    fid[wv][oc] = idc;
                }
            }
        }
        wave_sync();
        // ---- output slot of each candidate
        int octmask = 0;
#pragma unroll
        for (int o = 0; o < 8; ++o)
            if (fid[wv][o] >= 0) octmask |= 1 << o;
        const int n_oct = __popc(octmask);
#pragma unroll
        for (int q = 0; q < PER_LANE; ++q) {
            const int c = lane + 64 * q;
            if (c >= nc) continue;
            const double rc = sr2[wv][c];
            const int32_t kc = sid[wv][c];
            const int32_t idc = kc & 0x0FFFFFFF;
            const int oc = (kc >> 28) & 7;
            int slot;
            if (ork[q] == 0) {
                slot = __popc(octmask & ((1 << oc) - 1));
            } else {
                int fl = 0;
#pragma unroll
                for (int o = 0; o < 8; ++o)
                    if (fid[wv][o] >= 0 && key_less(fr2[wv][o], fid[wv][o], rc, idc)) ++fl;
                slot = n_oct + rk[q] - fl;
            }
            if (slot < m_max) v.hsten[(int64_t)slot * n + i] = idc;
        }
        if (lane == 0) v.rec[REC_M * n + i] = nc < m_max ? nc : m_max;
        wave_sync();
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
    for_candidates(v, g, i, [&](const Pt&, double, double, double, double) { ++nc; });
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
        int64_t vv = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += vv;
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
    for_candidates(v, g, i, [&](const Pt& p, double, double, double, double) {
        int q = nc++;
        while (q > 0 && out[q - 1] > p.id) {
            out[q] = out[q - 1];
            --q;
        }
        out[q] = p.id;
    });
}

__global__ void k_export_stencils(View v, int32_t* cnt_out, int32_t* idx_out,
                                  uint8_t* gm_out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= v.n) return;
    const GridInfo& g = v.grid[sys_of(v.off, v.n_sys, i)];
    const Rec r = load_rec(v, i);
    const int mm = v.m_max;
    if (gm_out) gm_out[i] = (uint8_t)r.gm;
    int m = 0;
    int32_t* out = idx_out ? idx_out + i * mm : nullptr;
    visit_stencil(v, g, i, r, [&](const Pt& p, double, double, double) {
        if (out && m < mm) {
            int q = m;
            while (q > 0 && out[q - 1] > p.id) {
                out[q] = out[q - 1];
                --q;
            }
            out[q] = p.id;
        }
        ++m;
    });
    if (out)
        for (int k = m; k < mm; ++k) out[k] = -1;
    if (cnt_out) cnt_out[i] = m;
}

// ---- tile map: the distinct list sources of each tile ------------------
//
// One block per tile of BLOCK consecutive particles.  The sources of all
// list entries of the tile are inserted in an LDS hash set, compacted,
// sorted ascending (bitonic, SORT_N keys) and stored; every list entry
// then gets the slot of its source in that order (a 16-bit word, with
// SLOT_MIRROR for a mirror entry).  A tile with more than STAGE_CAP
// sources, or whose hash set fills, is marked -1 (not staged).

constexpr int HASH_SIZE = 4096;        // LDS hash slots per tile (power of 2)
constexpr int SORT_N = 2048;           // keys sorted per tile (>= STAGE_CAP)
static_assert(STAGE_CAP <= SORT_N && SORT_N <= HASH_SIZE && SORT_N % BLOCK == 0 &&
                  HASH_SIZE % BLOCK == 0, "tile map sizes");
static_assert(STAGE_CAP <= (int)SLOT_MIRROR, "slots fit below the mirror bit");

__device__ __forceinline__ uint32_t src_hash(int32_t j)
{
    return ((uint32_t)j * 2654435761u) >> 20;   // top 12 bits: HASH_SIZE
}

// hash slot holding key j (present), found within HASH_SIZE probes
__device__ __forceinline__ int hash_find(const int32_t* hkey, int32_t j)
{
    uint32_t h = src_hash(j);
    for (int probe = 0; probe < HASH_SIZE; ++probe) {
        if (hkey[h] == j) return (int)h;
        h = (h + 1) & (HASH_SIZE - 1);
    }
    return -1;
}

__global__ __launch_bounds__(BLOCK) void k_tile_map(
    int64_t n, const int32_t* __restrict__ vl, const int32_t* __restrict__ vcnt,
    int32_t* __restrict__ tile_src, int32_t* __restrict__ tile_cnt,
    uint16_t* __restrict__ vs, int disable, const int32_t* gate)
{
    static_assert(HASH_SIZE == 1 << 12, "src_hash keeps 12 bits");
    if (gate && *gate == 0) return;
    // hkey: the set's keys, then (once sorted) each key's slot in the set
    __shared__ int32_t hkey[HASH_SIZE];
    __shared__ int32_t keys[SORT_N];
    __shared__ uint32_t wsum[BLOCK / 64];
    __shared__ int full;
    const int t = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t i = tile * BLOCK + t;
    const int cnt = i < n ? vcnt[i] : 0;
    for (int h = t; h < HASH_SIZE; h += BLOCK) hkey[h] = -1;
    if (t == 0) full = disable;
    __syncthreads();
    // list words are loaded MAP_BATCH at a time (one memory latency per
    // batch instead of per entry)
    constexpr int MAP_BATCH = 8;
    for (int k0 = 0; k0 < cnt; k0 += MAP_BATCH) {
        // a full set ends the insertions (the tile is not staged)
        if (*(volatile int*)&full) break;
        int32_t jb[MAP_BATCH];
        vl_load(vl, n, i, k0, jb);
#pragma unroll
        for (int u = 0; u < MAP_BATCH; ++u) {
            if (k0 + u >= cnt) continue;
            const int32_t j = jb[u] & ~MBIT;
            uint32_t h = src_hash(j);
            int probe = 0;
            for (; probe < HASH_SIZE; ++probe) {
                const int32_t old = atomicCAS(&hkey[h], -1, j);
                if (old == -1 || old == j) break;
                h = (h + 1) & (HASH_SIZE - 1);
            }
            if (probe == HASH_SIZE) full = 1;
            // the entry's hash slot (and mirror bit) until its source's
            // place in the sorted set is known
            vs[(int64_t)(k0 + u) * n + i] =
                (uint16_t)(h | ((jb[u] & MBIT) ? SLOT_MIRROR : 0u));
        }
    }
    __syncthreads();
    // compact: thread t takes hash slots [t PER, (t + 1) PER)
    constexpr int PER = HASH_SIZE / BLOCK;
    uint32_t mine = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) mine += hkey[t * PER + q] >= 0 ? 1u : 0u;
    uint32_t total = 0;
    uint32_t at = block_excl_scan(mine, wsum, total);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int32_t j = hkey[t * PER + q];
        if (j >= 0) {
            if (at < (uint32_t)SORT_N) keys[at] = j;
            ++at;
        }
    }
    const int S = (int)total;
    if (full || S > STAGE_CAP) {
        if (t == 0) tile_cnt[tile] = -1;
        return;
    }
    for (int q = S + t; q < SORT_N; q += BLOCK) keys[q] = INT32_MAX;
    __syncthreads();
    for (int size = 2; size <= SORT_N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int q = t; q < SORT_N / 2; q += BLOCK) {
                const int lo = 2 * q - (q & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int32_t a = keys[lo], b = keys[hi];
                if ((a > b) == up) {
                    keys[lo] = b;
                    keys[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    // every key's hash slot is found before any slot is overwritten
    constexpr int QPT = SORT_N / BLOCK;
    int hq[QPT];
#pragma unroll
    for (int r = 0; r < QPT; ++r) {
        const int q = t + r * BLOCK;
        hq[r] = -1;
        if (q < S) {
            tile_src[tile * STAGE_CAP + q] = keys[q];
            hq[r] = hash_find(hkey, keys[q]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < QPT; ++r)
        if (hq[r] >= 0) hkey[hq[r]] = t + r * BLOCK;
    if (t == 0) tile_cnt[tile] = S;
    __syncthreads();
    // hash slots -> slots in the sorted set (the thread rereads its own
    // words)
    for (int k0 = 0; k0 < cnt; k0 += MAP_BATCH) {
        uint32_t hb[MAP_BATCH];
#pragma unroll
        for (int u = 0; u < MAP_BATCH; ++u)
            hb[u] = k0 + u < cnt ? vs[(int64_t)(k0 + u) * n + i] : 0u;
#pragma unroll
        for (int u = 0; u < MAP_BATCH; ++u) {
            if (k0 + u >= cnt) continue;
            const uint32_t q = (uint32_t)hkey[hb[u] & (HASH_SIZE - 1)];
            vs[(int64_t)(k0 + u) * n + i] = (uint16_t)(q | (hb[u] & SLOT_MIRROR));
        }
    }
}

// 32-byte position records (x, y, z, 0) of the state the stencils are
// built on; every neighbour gather of the selection and the fits reads
// them (one cache line per neighbour instead of three).
__global__ __launch_bounds__(BLOCK) void k_pack_pos(int64_t n, const double* x,
                                                    const double* y, const double* z,
                                                    double* p4)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double2* r = reinterpret_cast<double2*>(p4 + 4 * i);
    r[0] = make_double2(x[i], y[i]);
    r[1] = make_double2(z[i], 0.0);
}

}  // namespace

lp_status list_build(lp_ctx* c, const int32_t* gate)
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (!gate) c->list_ok = false;
    if (n > 0 && (c->cfg.debug_flags & LP_DEBUG_PARTICLE_LIST)) {
        // the per-particle scan (same lists; kept to check the cell scan)
        if (c->periodic)
            hipLaunchKernelGGL(k_list_build<true>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, n, c->n_sys, w.off, w.grid, w.sst[0], w.sst[1],
                               w.sst[2], w.p4, w.cs, w.ce, w.vl, w.vcnt, w.err, gate);
        else
            hipLaunchKernelGGL(k_list_build<false>, dim3(blocks_for(n)), dim3(BLOCK), 0,
                               c->stream, n, c->n_sys, w.off, w.grid, w.sst[0], w.sst[1],
                               w.sst[2], w.p4, w.cs, w.ce, w.vl, w.vcnt, w.err, gate);
    } else if (n > 0) {
        // a wavefront per cell: the eager build knows the cell count; a
        // gated build reads it on the device and strides over the tables
        // with a grid sized by the particle count
        const int64_t tc = gate ? w.cells_max : c->total_cells;
        const int64_t* tdev = gate ? &w.summary->total_cells : nullptr;
        const int64_t groups = (tc + LC_WAVES - 1) / LC_WAVES;
        const int64_t cap = gate ? 2 * (int64_t)blocks_for(n) : (int64_t)LC_MAX_BLOCKS;
        const unsigned nb = (unsigned)std::max<int64_t>(1, std::min(groups, cap));
        if (c->periodic)
            hipLaunchKernelGGL(k_list_cells<true>, dim3(nb), dim3(BLOCK), 0, c->stream, n,
                               c->n_sys, w.grid, w.p4, w.cs, w.ce, tc, tdev, w.vl, w.vcnt,
                               w.err, gate);
        else
            hipLaunchKernelGGL(k_list_cells<false>, dim3(nb), dim3(BLOCK), 0, c->stream, n,
                               c->n_sys, w.grid, w.p4, w.cs, w.ce, tc, tdev, w.vl, w.vcnt,
                               w.err, gate);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "list build launch");
    c->list_ok = true;
    ++c->list_gen;
    // an eager build leaves the tile map stale (captured steps rebuild the
    // map under the same gate right after the list)
    if (!gate) c->map_ok = false;
    return LP_OK;
}

lp_status tile_map_build(lp_ctx* c, const int32_t* gate)
{
    Work& w = c->w;
    const int64_t n = c->n;
    if (!c->list_ok) {
        c->err = "the neighbour list has not been built";
        return LP_E_STATE;
    }
    if (n > 0)
        hipLaunchKernelGGL(k_tile_map, dim3(blocks_for(n)), dim3(BLOCK), 0, c->stream,
                           n, w.vl, w.vcnt, w.tile_src, w.tile_cnt, w.vs,
                           (c->cfg.debug_flags & LP_DEBUG_GLOBAL_GATHER) ? 1 : 0, gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "tile map launch");
    c->map_ok = true;
    return LP_OK;
}

lp_status stencils_build(lp_ctx* c, const double* const st[7], bool packed, int part)
{
    Work& w = c->w;
    const int64_t n = c->n;
    c->stencils_ok = false;
    if (!c->list_ok) {
        c->err = "the neighbour list has not been built";
        return LP_E_STATE;
    }
    View v = make_view(c, st);
    hipStream_t s = c->stream;
    if (n > 0 && part != STENCIL_TAIL) {
        // (the state copy or the re-sort of a step has packed them already)
        if (!packed)
            hipLaunchKernelGGL(k_pack_pos, dim3(blocks_for(n)), dim3(BLOCK), 0, s, n, st[0],
                               st[1], st[2], w.p4);
        // mirrors of the current state (ids n + k in ascending source order)
        const int64_t nb = (n + SORT_TILE - 1) / SORT_TILE;
        hipLaunchKernelGGL(k_mirror_count, dim3((unsigned)nb), dim3(BLOCK), 0, s, n,
                           c->n_sys, w.off, w.grid, st[2], w.bsum, w.hard_n, w.redo_n,
                           w.summary);
        // up to MIRROR_SUM_BLOCKS blocks each add the counts before them
        // (at most that many words per block, from L2) instead of a scan
        const int scanned =
            (nb > MIRROR_SUM_BLOCKS || (c->cfg.debug_flags & LP_DEBUG_MIRROR_SCAN)) ? 1 : 0;
        if (scanned)
            hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1024), 0, s,
                               (uint32_t*)w.bsum, nb, &w.summary->n_mirror);
        hipLaunchKernelGGL(k_mirror_write, dim3((unsigned)nb), dim3(BLOCK), 0, s, n,
                           c->n_sys, w.off, w.grid, w.bsum, scanned, &w.summary->n_mirror,
                           st[2], w.mirror_of, w.msrc);
        const int force = (c->cfg.debug_flags & LP_DEBUG_SORTED_STENCIL) ? 1 : 0;
        // the select phase times the selection kernel alone
        prof_mark(c, 1, false);
        if (c->periodic)
            hipLaunchKernelGGL(k_select<true>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, v,
                               w.hard, w.hard_n, force);
        else
            hipLaunchKernelGGL(k_select<false>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, v,
                               w.hard, w.hard_n, force);
        prof_mark(c, 1, true);
    }
    if (n > 0 && part != STENCIL_HEAD) {
        prof_mark(c, 2, false);
        hipLaunchKernelGGL(k_select_sorted, dim3(HARD_BLOCKS), dim3(BLOCK), 0, s, v,
                           w.hard, w.hard_n, w.err, w.cnt);
        prof_mark(c, 2, true);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "stencil launch");
    if (part != STENCIL_HEAD) c->stencils_ok = true;
    // k_mirror_count cleared the refit list and the displacement maximum
    if (n > 0 && part != STENCIL_TAIL) c->redo_clear = c->disp_clear = true;
    return LP_OK;
}

lp_status stencils_export(lp_ctx* c, const double* const st[7],
                          int64_t* cand_off, int32_t* cand_idx, int64_t cap,
                          int64_t* needed, int32_t* sten_cnt,
                          int32_t* sten_idx, uint8_t* ghost_mask,
                          int64_t* n_mirror)
{
    Work& w = c->w;
    const int64_t n = c->n;
    View v = make_view(c, st);
    hipStream_t s = c->stream;
    if (n_mirror) {
        hipError_t e = hipMemcpyAsync(w.h_summary, w.summary, sizeof(Summary),
                                      hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(c, e, "mirror count");
        *n_mirror = w.h_summary->n_mirror;
        c->n_mirror = *n_mirror;
    }
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
    if ((sten_cnt || sten_idx || ghost_mask) && n > 0)
        hipLaunchKernelGGL(k_export_stencils, dim3(blocks_for(n)), dim3(BLOCK), 0,
                           s, v, sten_cnt, sten_idx, ghost_mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "export launch");
    return LP_OK;
}

}  // namespace lp
