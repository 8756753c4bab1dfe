// Internal declarations of the LP granular-step library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "lp.h"

namespace lp {

constexpr int NCOEF = 9;          // unknowns of the 2nd-order 3D fit
constexpr int MMAX_LIMIT = 64;    // largest supported stencil cap
constexpr int MAXROWS = MMAX_LIMIT + 8;
constexpr int HIST_BUCKETS = 64;  // r^2 histogram of the stencil selection
#ifndef LP_LIST_CAP
#define LP_LIST_CAP 16
#endif
constexpr int LIST_CAP = LP_LIST_CAP;  // cut-bucket members ranked per thread
constexpr int VCAP = 256;         // neighbour-list entries per particle
constexpr int MASK_WORDS = VCAP / 64;  // keep bitmask words per particle
// Neighbour-list layout: a particle's entries come in chunks of VCHUNK
// consecutive entries (32 bytes, one cache sector), chunk c of every
// particle before chunk c + 1.  A thread appending entries fills one
// sector at a time, and reads entries k0 .. k0 + 7 (k0 a multiple of 8)
// as two 16-byte loads.
constexpr int VCHUNK = 8;
__host__ __device__ __forceinline__ int64_t vl_at(int64_t n, int64_t i, int k)
{
    return ((int64_t)(k / VCHUNK) * n + i) * VCHUNK + (k % VCHUNK);
}
// Entries k0 .. k0 + U - 1 of particle i (U a multiple of 4 dividing
// VCHUNK, k0 a multiple of U): U / 4 loads of 16 bytes.
template <int U>
__device__ __forceinline__ void vl_load(const int32_t* vl, int64_t n, int64_t i, int k0,
                                        int32_t (&e)[U])
{
    static_assert(U % 4 == 0 && VCHUNK % U == 0, "whole 16-byte words of one chunk");
    const int4* q = reinterpret_cast<const int4*>(vl + vl_at(n, i, k0));
#pragma unroll
    for (int w = 0; w < U / 4; ++w) {
        const int4 a = q[w];
        e[4 * w] = a.x;
        e[4 * w + 1] = a.y;
        e[4 * w + 2] = a.z;
        e[4 * w + 3] = a.w;
    }
}
// A tile is BLOCK consecutive particles.  The fits stage the fields of the
// distinct sources of a tile's neighbour lists in LDS (at most STAGE_CAP
// of them); a list entry names its source's slot in a 16-bit word whose
// top bit marks a mirror entry.
#ifndef LP_STAGE_CAP
#define LP_STAGE_CAP 1664
#endif
constexpr int STAGE_CAP = LP_STAGE_CAP;
constexpr uint32_t SLOT_MIRROR = 0x8000u;
constexpr int32_t MBIT = 0x40000000;  // list entry: mirror of the real id
constexpr int32_t NOID = 0x7FFFFFFF;
// per-particle stencil record (int32 fields, field f of particle i at
// f*n + i): kept rows, ghost mask, mode; the kept list entries themselves
// are a bitmask over the particle's neighbour list (word q at q*n + i)
constexpr int REC_M = 0, REC_GM = 1, REC_MODE = 2, REC_FIELDS = 3;
constexpr int MODE_ALL = 1, MODE_SORTED = 8;
constexpr uint8_t NO_CAND = 0xFF; // key code of a list entry outside R
constexpr int HARD_CAP = 256;     // candidates the sorted stencil path holds
constexpr int HARD_BLOCKS = 1024; // blocks of the sorted path (a wave per particle)
constexpr int HAND = 37;          // pass-1 -> pass-2 handoff doubles
// stencil size classes of the fits (rows, ghosts included): at most 16,
// at most 32, more
constexpr int NCLASS = 3;
constexpr int CLASS_ROWS0 = 16, CLASS_ROWS1 = 32;
constexpr int BLOCK = 256;        // threads per block of per-particle kernels
constexpr int SORT_ITEMS = 16;    // keys per thread in a radix tile
constexpr int RADIX_MAX_BITS = 9; // digit width of the radix sort, at most
constexpr int RADIX_MAX_DIGITS = 1 << RADIX_MAX_BITS;
constexpr int SORT_TILE = BLOCK * SORT_ITEMS;
// mirror numbering without a separate scan up to this many tiles
constexpr int MIRROR_SUM_BLOCKS = 2048;

// flag bits per particle
constexpr uint8_t FLAG_LINEAR = 1;
constexpr uint8_t FLAG_QR = 8;
constexpr uint8_t FLAG_QUAD = 16;       // a cubic fit fell back to the quadratic one

// device error codes (bit set in the error word)
constexpr int ERR_CAPACITY = 1;
constexpr int ERR_NUMERIC = 2;
constexpr int ERR_LIST = 4;       // a predictor stage left the neighbour list
constexpr int ERR_BOX = 8;        // a position lies beyond one period of its box

// Per-system grid, built on the device from the bounding box.
struct GridInfo {
    double x0, y0, z0, inv_c;   // origin, 1 / cell edge
    double inv_cx, inv_cy;      // 1 / cell edge along x, y (periodic: n / L)
    double xlo, ylo, Lx, Ly;    // periodic box (L = 0: open axis)
    double hLx, hLy;            // L / 2
    double R2, h, inv_h, R, wall;
    double Rv, Rv2;             // list radius R (1 + skin) and its square
    double inv_skin2;           // 1 / (skin R)^2 (0 when skin = 0)
    int64_t cell_base;          // first cell of this system in the tables
    int64_t pbeg, pend;         // particle range
    int32_t nx, ny, nz, pad;
};

// Small block read back by the host after the grid is built.
// Ordered encoding (see the displacement check) of +0.0: the starting
// value of the displacement maximum.
constexpr unsigned long long DISP_ZERO = 0x8000000000000000ull;

struct Summary {
    int64_t total_cells;
    int64_t n_mirror;
    int32_t axis_bits;
    int32_t bad;                // a cell coordinate needs more than 16 bits
    unsigned long long disp;    // ordered encoding of max (displacement/skin)^2
};

// Device error word.
struct ErrWord {
    int32_t code;
    int32_t pad;
    unsigned long long index;   // smallest offending particle
};

// Diagnostic counters (device).
struct Counters {
    unsigned long long qr_refits;
    unsigned long long hard_stencils;
    unsigned long long below_wall;
    unsigned long long rebuilds;    // list rebuilds decided on the device
    unsigned long long pad[4];
};

// Everything a per-particle kernel needs to find neighbours and states.
struct View {
    int64_t n;                  // real particles
    int32_t n_sys;
    int32_t m_max;
    const int64_t* off;         // system offsets (device)
    const lp_params* prm;
    const GridInfo* grid;
    // real particles in cell order (current positions)
    const double *x, *y, *z, *u, *v, *w, *V;
    // the same positions as 32-byte records (x, y, z, 0), packed when the
    // stencils are built: one neighbour's position is one cache line
    const double* p4;
    // mirrors: mirror_of[j] = k (mirror id n + k) or -1; msrc[k] = j
    const int32_t* mirror_of;
    const int32_t* msrc;
    // neighbour list with skin (entry k of particle i at vl_at(n, i, k))
    const int32_t* vl;
    const int32_t* vcnt;
    // per tile: its list sources in ascending order (STAGE_CAP per tile)
    // and their count (-1: not staged); slot of every list entry
    const int32_t* tile_src;
    const int32_t* tile_cnt;
    const uint16_t* vs;
    uint32_t* code;             // r^2 buckets of the list entries, four per word
                                // (entry k: byte k % 4 of word (k / 4) n + i;
                                // NO_CAND: outside R)
    // stencil records, keep bitmasks and explicit stencils of the sorted path
    int32_t* rec;
    uint64_t* kmask;            // MASK_WORDS x n
    int32_t* hsten;             // m_max x n
    double ghost_margin;
    double fallback_tol;
    double redo_ratio;          // Gram pivot ratio that triggers a QR refit
    int32_t weight;
    int32_t debug;
    int32_t wall_pressure;      // hydrostatic mirror pressure
    int32_t periodic;           // some system has a periodic axis
    int32_t min_real;           // fewer real stencil rows: linear fit
};

struct Work {
    int64_t n_max = 0, cells_max = 0;
    int32_t m_max = 0;
    // systems
    int64_t* off = nullptr;
    lp_params* prm = nullptr;
    GridInfo* grid = nullptr;
    unsigned long long* bbox = nullptr;   // n_sys x 6 ordered encodings
    Summary* summary = nullptr;
    Summary* h_summary = nullptr;         // pinned host copy
    ErrWord* err = nullptr;
    Counters* cnt = nullptr;
    // sort
    unsigned long long *keys0 = nullptr, *keys1 = nullptr;
    int32_t *vals0 = nullptr, *vals1 = nullptr;
    uint32_t* hist = nullptr;
    int64_t hist_cap = 0;
    // working copy of the state (cell order)
    double* sst[7] = {nullptr};
    double* p4 = nullptr;                 // 4 x n: x y z 0 of the stencils' state
    double* xref[3] = {nullptr};          // positions at the last list build
    // mirrors
    int32_t* mirror_of = nullptr;
    int32_t* msrc = nullptr;
    int32_t* bsum = nullptr;              // scan block sums
    // cell tables
    int32_t *cs = nullptr, *ce = nullptr;
    // neighbour list, records, sorted-path stencils
    int32_t* vl = nullptr;
    int32_t* vcnt = nullptr;
    int32_t* tile_src = nullptr;          // tiles x STAGE_CAP
    int32_t* tile_cnt = nullptr;          // tiles
    uint16_t* vs = nullptr;               // VCAP x n
    uint32_t* code = nullptr;             // VCAP / 4 x n
    int32_t* rec = nullptr;
    uint64_t* kmask = nullptr;            // MASK_WORDS x n
    int32_t* hsten = nullptr;
    int32_t* hard = nullptr;
    unsigned int* hard_n = nullptr;
    // fits
    int32_t* redo = nullptr;
    unsigned int* redo_n = nullptr;
    double *P = nullptr, *eta = nullptr;
    double* hand = nullptr;               // HAND x n
    float* uf = nullptr;                  // 45 x n float32 factors (refined mode)
    // adjoint
    double* adj[7] = {nullptr};           // state cotangent accumulators
    double* adj_P = nullptr;
    double* adj_E = nullptr;
    double* adj_stash = nullptr;          // 11 x n
    double* coefu = nullptr;              // 27 x n forward velocity coefficients
    int32_t* adj_perm = nullptr;
    double* adj_recv = nullptr;           // 6 x n: cotangents received from neighbours
    double* adj_M = nullptr;              // 31 x n: Gram moments of the stencils
    // captured step sequences
    int32_t* gate = nullptr;              // [0] rebuild, [1] keep
    // second-order steps: predictor state and its right-hand side
    double* sst2[7] = {nullptr};
    double* acc2 = nullptr;               // 3 x n
    double* dVdt2 = nullptr;
    double* adj2[7] = {nullptr};          // cotangent of the predictor state
    int32_t* ids_tmp = nullptr;
    double* acc = nullptr;                // 3 x n
    double* dVdt = nullptr;
    uint8_t* flags = nullptr;
    // stencil size classes: particles of class c at cls_idx[c n ...],
    // their count in cls_cnt[c]
    int32_t* cls_idx = nullptr;
    uint32_t* cls_cnt = nullptr;
    // export helpers
    int64_t* coff = nullptr;
};

// Every workspace buffer and its element count, in one place.  A(p, count)
// receives each buffer pointer; lp_reserve allocates them, the
// allocation-free step carves them from a static device array.  With
// forward_only, the buffers only the adjoints, the second-order step,
// captured steps and the candidate export use are left out (null).
template <class F>
constexpr void work_layout(Work& w, int64_t n_max, int64_t cells_max, int mm,
                           int sys_cap, bool forward_only, F&& A)
{
    const int64_t nb = (n_max + SORT_TILE - 1) / SORT_TILE;
    const int64_t tiles = (n_max + BLOCK - 1) / BLOCK;
    A(w.off, sys_cap + 1); A(w.prm, sys_cap); A(w.grid, sys_cap);
    A(w.bbox, 6 * sys_cap); A(w.summary, 1); A(w.err, 1); A(w.cnt, 1);
    A(w.keys0, n_max); A(w.keys1, n_max); A(w.vals0, n_max); A(w.vals1, n_max);
    A(w.hist, RADIX_MAX_DIGITS * nb);
    for (int a = 0; a < 7; ++a) A(w.sst[a], n_max);
    A(w.p4, 4 * n_max);
    for (int a = 0; a < 3; ++a) A(w.xref[a], n_max);
    A(w.mirror_of, n_max); A(w.msrc, n_max); A(w.bsum, nb + 1);
    A(w.cs, cells_max); A(w.ce, cells_max);
    A(w.vl, (int64_t)VCAP * n_max); A(w.vcnt, n_max);
    A(w.tile_src, (int64_t)STAGE_CAP * tiles);
    A(w.tile_cnt, tiles);
    A(w.vs, (int64_t)VCAP * n_max);
    A(w.code, (int64_t)(VCAP / 4) * n_max);
    A(w.kmask, (int64_t)MASK_WORDS * n_max);
    A(w.rec, (int64_t)REC_FIELDS * n_max); A(w.hsten, (int64_t)mm * n_max);
    A(w.hard, n_max); A(w.hard_n, 1);
    A(w.redo, n_max); A(w.redo_n, 1);
    A(w.P, n_max); A(w.eta, n_max); A(w.hand, (int64_t)HAND * n_max);
    A(w.uf, (int64_t)45 * n_max);
    A(w.acc, 3 * n_max); A(w.dVdt, n_max); A(w.flags, n_max);
    A(w.cls_idx, NCLASS * n_max); A(w.cls_cnt, 4);
    if (forward_only) return;
    for (int a = 0; a < 7; ++a) A(w.adj[a], n_max);
    A(w.adj_P, n_max); A(w.adj_E, n_max); A(w.adj_stash, (int64_t)11 * n_max);
    A(w.coefu, (int64_t)27 * n_max); A(w.adj_perm, n_max);
    A(w.adj_recv, 6 * n_max);
    A(w.adj_M, (int64_t)31 * n_max);
    A(w.gate, 4); A(w.ids_tmp, n_max);
    for (int a = 0; a < 7; ++a) A(w.sst2[a], n_max);
    for (int a = 0; a < 7; ++a) A(w.adj2[a], n_max);
    A(w.acc2, 3 * n_max); A(w.dVdt2, n_max);
    A(w.coff, n_max + 1);
}

}  // namespace lp

struct lp_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    lp_config cfg{};
    int32_t n_sys = 0;
    int64_t n = 0;
    std::vector<int64_t> h_off;
    std::vector<lp_params> h_prm;
    bool periodic = false;                // some system has a periodic axis
    bool map_ok = false;                  // the tile map matches the current list
    lp::Work w;
    int axis_bits = 0;
    int64_t total_cells = 0;
    int64_t n_mirror = 0;
    bool list_ok = false;       // neighbour list valid for the working state
    int64_t list_gen = 0;       // generation of the current list (one per build)
    int lpp1 = 1, lpp2 = 1;     // lanes per particle of the two fit kernels
    // size-class dispatch of the fits (lp_autotune, LP_DEBUG_CLASSES):
    // lanes per particle of each class in each fit, and what the last
    // autotune measured (class counts, best milliseconds)
    bool classes = false;
    // (lanes 0 on the largest class: the LDS-staged one-lane tile kernel)
    int cls_lpp1[lp::NCLASS] = {1, 2, 4}, cls_lpp2[lp::NCLASS] = {1, 2, 4};
    int64_t cls_count[lp::NCLASS] = {0, 0, 0};
    double tune_ms[8] = {0};
    int64_t rebuilds = 0;       // list rebuilds since the last lp_stats
    // the work enqueued last left the fits' refit counter (redo_clear) or
    // the displacement maximum (disp_clear) at zero, so the next user
    // need not clear it (set by a stencil build, taken by the next user)
    bool redo_clear = false, disp_clear = false;
    // the displacement check's maximum, copied to the host behind this
    // event (list_check_start), not yet read (list_check_wait)
    hipEvent_t chk_ev = nullptr;
    bool chk_pending = false;
    // phase timing (lp_profile)
    bool prof = false;
    hipEvent_t ev[16] = {nullptr};
    double prof_ms[8] = {0};
    int64_t prof_steps = 0;
    // call-order state: the cell build and stencils refer to this state
    const double* built_x = nullptr;
    bool cells_ok = false;
    bool stencils_ok = false;
    // side stream of an eager step that rebuilt its list: the tile map is
    // built there while the step's own stream runs the mirrors and the
    // selection, which do not read it; the fits wait for map_join
    hipStream_t map_stream = nullptr;
    hipEvent_t map_fork = nullptr, map_join = nullptr;
    bool map_side = true;       // false: the allocation-free step's context
                                // (which creates no stream) builds it in line
    // captured step sequence (lp_step_graph) and what it was captured for
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        const double* st[7];
        const int32_t* ids;
        double dt;
        int32_t nsteps, bits;
        int64_t n;
        int32_t n_sys;
        bool operator==(const GraphKey& o) const
        {
            for (int a = 0; a < 7; ++a)
                if (st[a] != o.st[a]) return false;
            return ids == o.ids && dt == o.dt && nsteps == o.nsteps && bits == o.bits &&
                   n == o.n && n_sys == o.n_sys;
        }
    } gkey{};
    std::string err;
};

namespace lp {

// ---- device helpers -------------------------------------------------

// Logical block index that gives each XCD a contiguous range of blocks.
// Blocks are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8); remapping keeps neighbouring particles (and their shared
// neighbour data) in one XCD's L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t q = nb >> 3, r = nb & 7;
    const int64_t x = b & 7, t = b >> 3;
    return x * q + (x < r ? x : r) + t;
}

__device__ __forceinline__ int sys_of(const int64_t* off, int n_sys, int64_t i)
{
    int lo = 0, hi = n_sys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// bit k of the low 16 bits of x -> bit 3k
__device__ __forceinline__ uint64_t spread3_64(uint64_t x)
{
    x &= 0xFFFFull;
    x = (x | (x << 16)) & 0x0000FF0000FFull;
    x = (x | (x << 8)) & 0x00F00F00F00Full;
    x = (x | (x << 4)) & 0x0C30C30C30C3ull;
    x = (x | (x << 2)) & 0x249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t morton3(uint32_t cx, uint32_t cy, uint32_t cz)
{
    return spread3_64(cx) | (spread3_64(cy) << 1) | (spread3_64(cz) << 2);
}

// Exact float64 operations: the integer decisions of the method (cell
// coordinates, candidate test, ordering keys) must round exactly as the
// plain float64 definition does, so these helpers forbid fused
// multiply-add contraction.
__device__ __forceinline__ double dsub(double a, double b)
{
#pragma clang fp contract(off)
    return a - b;
}
__device__ __forceinline__ double dmul(double a, double b)
{
#pragma clang fp contract(off)
    return a * b;
}
__device__ __forceinline__ double dadd(double a, double b)
{
#pragma clang fp contract(off)
    return a + b;
}

// Periodic axes (period L > 0; L = 0 leaves a coordinate unchanged): the
// copy of xj nearest to xi (xj - L when xj - xi > L/2, xj + L when below
// -L/2), and a coordinate within one period mapped into [lo, lo + L).
__device__ __forceinline__ double image_coord(double xj, double xi, double L, double hL)
{
    if (L > 0.0) {
        const double d = dsub(xj, xi);
        if (d > hL) return dsub(xj, L);
        if (d < -hL) return dadd(xj, L);
    }
    return xj;
}
__device__ __forceinline__ double wrap_coord(double x, double lo, double L)
{
    if (L > 0.0) {
        if (x >= dadd(lo, L)) return dsub(x, L);
        if (x < lo) return dadd(x, L);
    }
    return x;
}

// r^2 exactly as the method defines it: (dx*dx + dy*dy) + dz*dz, each
// product and sum rounded separately.
__device__ __forceinline__ double dist2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    const double xx = dx * dx;
    const double yy = dy * dy;
    const double zz = dz * dz;
    const double s = xx + yy;
    return s + zz;
}

__device__ __forceinline__ void raise_error(ErrWord* e, int code, int64_t idx)
{
    atomicOr(&e->code, code);
    atomicMin(&e->index, (unsigned long long)idx);
}

}  // namespace lp

// ---- host-side launchers (defined in the .hip files) -----------------
namespace lp {
// Morton sort of the input into the working copy, cell tables, neighbour
// list with skin and reference positions.
lp_status cells_build(lp_ctx* c, double* const st[7], int32_t* perm_out);
// Copies the input into the working copy in the same order (no rebuild);
// with arrays = false only the identity permutation is written.
lp_status state_copy(lp_ctx* c, double* const st[7], int32_t* perm_out,
                     const int32_t* gate = nullptr, bool arrays = true);
// Re-sort + list rebuild entirely on the device, skipped unless *gate;
// ids (optional) are permuted with the state; `bits` per grid axis.
lp_status cells_build_device(lp_ctx* c, double* const st[7], int32_t* ids,
                             const int32_t* gate, int bits);
// ids[i] = ids[perm[i]]
lp_status permute_ids(lp_ctx* c, const int32_t* perm, int32_t* ids);
// working copy of st in the order perm (sst[new] = st[perm[new]]; perm
// null: the same order) with its positions' 32-byte records
lp_status state_gather(lp_ctx* c, const double* const st[7], const int32_t* perm);
// Device-side rebuild decision into w.gate (no synchronisation).
lp_status rebuild_decision(lp_ctx* c, const double* const st[7], int force, bool first);
// Copies the working copy back into the caller's arrays.
lp_status state_write_back(lp_ctx* c, double* const out[7]);
// Largest displacement since the list build in units of the skin: the
// check enqueued with the state copied into the working copy (the 32-byte
// position records too), its result copied to the host behind an event,
// and the wait for that copy (the stream may run later work meanwhile).
// ratio < 0 when no list exists.
lp_status list_check_start(lp_ctx* c, const double* const st[7]);
lp_status list_check_wait(lp_ctx* c, double* ratio);
// Mirror ids of the current state, stencil records.
// packed: the positions' 32-byte records (p4) already hold st's positions
// (written by the step's state copy or re-sort).  part: STENCIL_ALL, or
// STENCIL_HEAD (mirrors and the histogram selection, which a step enqueues
// before it knows whether the list must be rebuilt) and then STENCIL_TAIL
// (the exact path for the particles the selection handed over).
enum { STENCIL_ALL = 0, STENCIL_HEAD = 1, STENCIL_TAIL = 2 };
lp_status stencils_build(lp_ctx* c, const double* const st[7], bool packed = false,
                         int part = STENCIL_ALL);
lp_status stencils_export(lp_ctx* c, const double* const st[7],
                          int64_t* cand_off, int32_t* cand_idx, int64_t cap,
                          int64_t* needed, int32_t* sten_cnt,
                          int32_t* sten_idx, uint8_t* ghost_mask,
                          int64_t* n_mirror);
lp_status list_build(lp_ctx* c, const int32_t* gate = nullptr);
// Tile map of the current list (the fits' LDS staging); skipped unless
// *gate when gate is given.  A new list leaves the fits on global
// gathers until this is called.
lp_status tile_map_build(lp_ctx* c, const int32_t* gate = nullptr);
lp_status fit_generic(lp_ctx* c, const double* const st[7], const double* f,
                      int k, const int32_t* msign, const int32_t* gzero,
                      double* coef, uint8_t* flags);
lp_status rhs_from_coef(lp_ctx* c, const double* const st[7],
                        const double* coef_u, double* dVdt, double* acc,
                        double* diag, double* grad, uint8_t* flags);
lp_status step_rhs(lp_ctx* c, const double* const st[7]);
// times each lanes-per-particle variant of the two fit kernels on the
// stencils of st and keeps the fastest (choice: host int32[2], optional)
lp_status autotune_fits(lp_ctx* c, const double* const st[7], int32_t* choice);
// pass 2 with acc / dVdt stored and, when out is given, the explicit
// update written to out (fp64: float64 kernels whatever the precision)
lp_status step_pass2(lp_ctx* c, const double* const st[7], double dt,
                     double* const out[7], double* acc, double* dVdt,
                     bool fp64 = false);
// predictor of the second-order step: w.sst2 = w.sst + dt (u, acc, dVdt)
// from w.acc / w.dVdt, with the device check that it stays within half
// the list skin (ERR_LIST)
lp_status heun_predictor(lp_ctx* c, double dt);
// second-order (Heun) step on the sorted working state (lp_step2), after
// pass 1 and pass 2 at w.sst
lp_status step_heun(lp_ctx* c, double dt, double* const out[7]);
// pass 1 in float64 with the velocity coefficients stored (adjoint input)
lp_status step_pass1_coef(lp_ctx* c, const double* const st[7]);
// Cotangent seeds of one reverse right-hand-side evaluation.  With
// N = nA A + nB B (B optional), the state accumulators start at
// iA A + iB B with c_ux N_(x,y,z) added to (u, v, w), and the cotangents of
// the acceleration and of dV/dt are c_a (N_(u,v,w) + k_x N_(x,y,z)) and
// c_d N_V.  One explicit step: A = lam, c_ux = c_a = c_d = dt, k_x = dt/2.
struct AdjSeed {
    const double* A[7] = {nullptr};
    const double* B[7] = {nullptr};
    double iA = 1.0, iB = 0.0, nA = 1.0, nB = 0.0;
    double c_ux = 0.0, c_a = 0.0, k_x = 0.0, c_d = 0.0;
};
// reverse of the right-hand side (and the update the seed describes) on
// the sorted state st (after stencils_build and step_pass1_coef on st);
// out: cotangent of the input in its order (perm[new] = old; perm null:
// st's order); dparams += parameter cotangents
lp_status step_adjoint(lp_ctx* c, const double* const st[7], const AdjSeed& seed,
                       double* const out[7], double* dparams, const int32_t* perm);
lp_status step_update(lp_ctx* c, const double* const st[7], double dt,
                      double* const out[7]);
View make_view(lp_ctx* c, const double* const st[7]);
// records the begin (end = false) or end event of phase `ph` when profiling
void prof_mark(lp_ctx* c, int ph, bool end);
lp_status hip_fail(lp_ctx* c, hipError_t e, const char* what);
}  // namespace lp
