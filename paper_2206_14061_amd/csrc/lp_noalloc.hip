// Allocation-free explicit step (lp_step_noalloc): one lp_step on a fresh
// context, with its forward-step workspace carved from a file-scope
// device array instead of memory that lp_reserve allocates.  For callers
// that cannot allocate device memory.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "lp_internal.h"

namespace lp {
namespace {

constexpr int64_t NOALLOC_N = 16384;        // particles (mirrors counted apart)
constexpr int64_t NOALLOC_CELLS = 65536;    // cells of all systems
constexpr int NOALLOC_SYS = 64;             // systems
constexpr int NOALLOC_DEVICES = 64;
constexpr int64_t ALIGN = 256;

constexpr int64_t align_up(int64_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

// bytes of the forward-step workspace at the limits above, each buffer
// aligned to 256 bytes
constexpr int64_t noalloc_bytes()
{
    Work w{};
    int64_t b = 0;
    work_layout(w, NOALLOC_N, NOALLOC_CELLS, MMAX_LIMIT, NOALLOC_SYS, true,
                [&b](auto*& p, int64_t cnt) {
                    using T = typename std::remove_reference<decltype(*p)>::type;
                    b = align_up(b) + (int64_t)sizeof(T) * (cnt > 0 ? cnt : 1);
                });
    return align_up(b);
}

constexpr int64_t SCRATCH_BYTES = noalloc_bytes();
static_assert(SCRATCH_BYTES < (64ll << 20), "the static workspace stays below 64 MiB");

// The workspace.  In host code this name is only a stand-in for the
// symbol: its device address comes from hipGetSymbolAddress, once per
// device.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Per device: the scratch address and a context whose workspace points
// into it (never freed; it lives as long as the process).
struct DevSlot {
    std::once_flag once;
    hipError_t init_err = hipSuccess;
    unsigned char* base = nullptr;
    lp_ctx* ctx = nullptr;
    Summary host_summary{};
};

DevSlot g_dev[NOALLOC_DEVICES];
std::mutex g_call_mutex[NOALLOC_DEVICES];

// Clears the words a call must start from: no latched error, zero
// counters and summary, no tile staged.
__global__ void k_noalloc_clear(ErrWord* err, Counters* cnt, Summary* sum,
                                int32_t* tile_cnt, int64_t tiles)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        err->code = 0;
        err->pad = 0;
        err->index = ~0ull;
        *cnt = Counters{};
        *sum = Summary{};
    }
    if (i < tiles) tile_cnt[i] = -1;
}

void init_slot(DevSlot& d)
{
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        d.init_err = e != hipSuccess ? e : hipErrorInvalidSymbol;
        return;
    }
    d.base = (unsigned char*)ptr;
    lp_ctx* c = new (std::nothrow) lp_ctx();
    if (!c) {
        d.init_err = hipErrorOutOfMemory;
        return;
    }
    Work& w = c->w;
    int64_t off = 0;
    work_layout(w, NOALLOC_N, NOALLOC_CELLS, MMAX_LIMIT, NOALLOC_SYS, true,
                [&](auto*& p, int64_t cnt) {
                    using T = typename std::remove_reference<decltype(*p)>::type;
                    off = align_up(off);
                    p = (T*)(d.base + off);
                    off += (int64_t)sizeof(T) * (cnt > 0 ? cnt : 1);
                });
    w.h_summary = &d.host_summary;
    w.n_max = NOALLOC_N;
    w.cells_max = NOALLOC_CELLS;
    w.m_max = MMAX_LIMIT;
    w.hist_cap = RADIX_MAX_DIGITS * ((NOALLOC_N + SORT_TILE - 1) / SORT_TILE);
    // no side stream for the tile map: this context creates no stream
    c->map_side = false;
    if (hipGetDevice(&c->device) != hipSuccess) {
        d.init_err = hipErrorInvalidDevice;
        delete c;
        return;
    }
    d.ctx = c;
}

}  // namespace
}  // namespace lp

using namespace lp;

extern "C" lp_status lp_step_noalloc(void* stream, const lp_config* cfg, int32_t n_sys,
                                     const int64_t* offsets, const lp_params* params,
                                     lp_state* s, double dt, int32_t* perm)
{
    if (!s || !offsets || !params || n_sys < 1 || !(dt > 0.0) || !std::isfinite(dt))
        return LP_E_ARG;
    if (n_sys > NOALLOC_SYS || offsets[0] != 0 || offsets[n_sys] < 0 ||
        offsets[n_sys] > NOALLOC_N)
        return offsets[0] != 0 || offsets[n_sys] < 0 ? LP_E_ARG : LP_E_CAPACITY;
    lp_config c0;
    lp_config_default(&c0);
    if (cfg) c0 = *cfg;
    if (c0.m_max < 1 || c0.m_max > MMAX_LIMIT || !(c0.cond_max > 1.0) ||
        !(c0.ghost_margin >= 0.0) || !(c0.fallback_tol >= 0.0) ||
        (c0.weight != LP_W_UNIT && c0.weight != LP_W_GAUSS) ||
        (c0.precision != LP_FP64 && c0.precision != LP_FP32_REFINED) ||
        !(c0.skin >= 0.0 && c0.skin <= 1.0) ||
        (c0.wall_reflect != 0 && c0.wall_reflect != 1) ||
        (c0.wall_pressure != 0 && c0.wall_pressure != 1) ||
        (c0.fit_order != 2 && c0.fit_order != 3) ||
        (c0.fit_order == 3 && c0.m_max > 56) ||
        c0.min_real_rows < 0 || c0.min_real_rows > MMAX_LIMIT)
        return LP_E_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_DEVICES)
        return LP_E_HIP;
    DevSlot& d = g_dev[dev];
    std::call_once(d.once, [&d] { init_slot(d); });
    if (d.init_err != hipSuccess || !d.ctx) return LP_E_HIP;
    std::lock_guard<std::mutex> lock(g_call_mutex[dev]);
    lp_ctx* c = d.ctx;
    c->stream = (hipStream_t)stream;
    c->cfg = c0;
    c->lpp1 = c->lpp2 = 1;
    if (c0.debug_flags & LP_DEBUG_LANES2) c->lpp1 = c->lpp2 = 2;
    if (c0.debug_flags & LP_DEBUG_LANES4) c->lpp1 = c->lpp2 = 4;
    c->prof = false;
    c->rebuilds = 0;
    lp_status r = lp_set_systems(c, n_sys, offsets, params);
    if (r != LP_OK) return r;
    // state left by the previous call on this device: none of it is kept
    const int64_t tiles = (NOALLOC_N + BLOCK - 1) / BLOCK;
    hipLaunchKernelGGL(k_noalloc_clear, dim3((unsigned)((tiles + BLOCK - 1) / BLOCK)),
                       dim3(BLOCK), 0, c->stream, c->w.err, c->w.cnt, c->w.summary,
                       c->w.tile_cnt, tiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "lp_step_noalloc clear");
    c->list_ok = c->map_ok = c->cells_ok = c->stencils_ok = false;
    c->redo_clear = c->disp_clear = false;
    c->built_x = nullptr;
    r = lp_step(c, s, dt, perm, nullptr);
    // device-side errors of this call (synchronises)
    const lp_status rs = lp_sync_status(c, nullptr);
    c->list_ok = c->map_ok = false;
    return r != LP_OK ? r : rs;
}
