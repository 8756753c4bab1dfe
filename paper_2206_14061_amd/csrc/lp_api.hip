// C ABI entry points, context and workspace of the LP granular-step library.
#include <cmath>
#include <vector>
#include <cstring>
#include <new>

#include "lp_internal.h"

namespace lp {

constexpr int SYS_CAP = 4096;

lp_status hip_fail(lp_ctx* c, hipError_t e, const char* what)
{
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return LP_E_HIP;
}

void prof_mark(lp_ctx* c, int ph, bool end)
{
    if (!c->prof) return;
    hipEventRecord(c->ev[2 * ph + (end ? 1 : 0)], c->stream);
}

View make_view(lp_ctx* c, const double* const st[7])
{
    Work& w = c->w;
    View v;
    v.n = c->n;
    v.n_sys = c->n_sys;
    v.m_max = c->cfg.m_max;
    v.off = w.off;
    v.prm = w.prm;
    v.grid = w.grid;
    v.x = st[0]; v.y = st[1]; v.z = st[2];
    v.u = st[3]; v.v = st[4]; v.w = st[5]; v.V = st[6];
    v.p4 = w.p4;
    v.mirror_of = w.mirror_of;
    v.msrc = w.msrc;
    v.vl = w.vl;
    v.vcnt = w.vcnt;
    v.tile_src = w.tile_src;
    v.tile_cnt = w.tile_cnt;
    v.vs = w.vs;
    v.code = w.code;
    v.rec = w.rec;
    v.kmask = w.kmask;
    v.hsten = w.hsten;
    v.ghost_margin = c->cfg.ghost_margin;
    v.fallback_tol = c->cfg.fallback_tol;
    v.redo_ratio = 1.0 / c->cfg.cond_max;
    v.weight = c->cfg.weight;
    v.debug = c->cfg.debug_flags;
    v.wall_pressure = c->cfg.wall_pressure;
    v.periodic = c->periodic ? 1 : 0;
    v.min_real = c->cfg.min_real_rows;
    return v;
}

namespace {

template <class T>
hipError_t alloc(T*& p, int64_t count)
{
    if (p) {
        hipFree(p);
        p = nullptr;
    }
    const size_t bytes = sizeof(T) * (size_t)(count > 0 ? count : 1);
    return hipMalloc((void**)&p, bytes);
}

void free_work(Work& w)
{
    auto f = [](auto*& p) {
        if (p) hipFree(p);
        p = nullptr;
    };
    f(w.off); f(w.prm); f(w.grid); f(w.bbox); f(w.summary); f(w.err); f(w.cnt);
    f(w.keys0); f(w.keys1); f(w.vals0); f(w.vals1); f(w.hist);
    for (int a = 0; a < 7; ++a) f(w.sst[a]);
    f(w.p4);
    for (int a = 0; a < 3; ++a) f(w.xref[a]);
    f(w.mirror_of); f(w.msrc); f(w.bsum); f(w.cs); f(w.ce);
    f(w.vl); f(w.vcnt); f(w.tile_src); f(w.tile_cnt); f(w.vs);
    f(w.code); f(w.rec); f(w.kmask); f(w.hsten); f(w.hard); f(w.hard_n);
    f(w.redo); f(w.redo_n);
    f(w.P); f(w.eta); f(w.hand); f(w.uf);
    for (int a = 0; a < 7; ++a) f(w.adj[a]);
    f(w.adj_P); f(w.adj_E); f(w.adj_stash); f(w.coefu); f(w.adj_perm);
    f(w.adj_recv); f(w.adj_M);
    f(w.gate); f(w.ids_tmp);
    for (int a = 0; a < 7; ++a) f(w.sst2[a]);
    for (int a = 0; a < 7; ++a) f(w.adj2[a]);
    f(w.acc2); f(w.dVdt2); f(w.acc); f(w.dVdt); f(w.flags); f(w.coff);
    f(w.cls_idx); f(w.cls_cnt);
    if (w.h_summary) hipHostFree(w.h_summary);
    w.h_summary = nullptr;
    w.n_max = w.cells_max = 0;
}

lp_status check_ready(lp_ctx* c, const lp_state* s)
{
    if (!c) return LP_E_ARG;
    if (c->w.n_max == 0) {
        c->err = "lp_reserve has not been called";
        return LP_E_STATE;
    }
    if (c->n_sys == 0) {
        c->err = "lp_set_systems has not been called";
        return LP_E_STATE;
    }
    if (c->n > c->w.n_max) {
        c->err = "systems hold " + std::to_string(c->n) + " particles, reserved " +
                 std::to_string(c->w.n_max);
        return LP_E_CAPACITY;
    }
    if (s) {
        const double* p[7] = {s->x, s->y, s->z, s->u, s->v, s->w, s->V};
        for (int a = 0; a < 7; ++a)
            if (!p[a] && c->n > 0) {
                c->err = "null state array";
                return LP_E_ARG;
            }
    }
    return LP_OK;
}

void state_arrays(const lp_state* s, double* st[7])
{
    st[0] = s->x; st[1] = s->y; st[2] = s->z;
    st[3] = s->u; st[4] = s->v; st[5] = s->w; st[6] = s->V;
}

void drop_graph(lp_ctx* c)
{
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    if (c->graph) hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

// perm copy on the context's stream
lp_status copy_perm(lp_ctx* c, const int32_t* src, int32_t* dst)
{
    if (!dst || src == dst || c->n == 0) return LP_OK;
    hipError_t e = hipMemcpyAsync(dst, src, sizeof(int32_t) * c->n,
                                  hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "permutation copy");
}

// Working copy of the state an adjoint differentiates, in the order of the
// step it reverses.  Without a record: re-sorted and a list built as by
// lp_build_cells (*order = that permutation).  With a record: the step's
// own order (*order = rec->perm, or null for the identity) and its list,
// which must still be current.
lp_status adjoint_order(lp_ctx* c, double* const in[7], const lp_step_record* rec,
                        const int32_t** order)
{
    if (!rec) {
        *order = c->w.adj_perm;
        return cells_build(c, in, c->w.adj_perm);
    }
    if (!c->list_ok || rec->list_gen != c->list_gen) {
        c->err = "the neighbour list of the recorded step is no longer current "
                 "(the list was rebuilt since): recompute the step";
        return LP_E_STATE;
    }
    const double* cin[7];
    for (int a = 0; a < 7; ++a) cin[a] = in[a];
    if (rec->resorted) {
        if (!rec->perm) {
            c->err = "a re-sorted step record needs its perm array";
            return LP_E_ARG;
        }
        *order = rec->perm;
        return state_gather(c, cin, rec->perm);
    }
    *order = nullptr;
    return state_gather(c, cin, nullptr);
}

// One step with no host synchronisation: device-side rebuild decision,
// gated re-sort + list rebuild or state copy, stencils, fits, update into
// the caller's arrays.
lp_status step_device(lp_ctx* c, double* const in[7], int32_t* ids, double dt, int bits,
                      bool first)
{
    const double* cin[7];
    for (int a = 0; a < 7; ++a) cin[a] = in[a];
    // the decision copies the state into the working state, which a
    // rebuild overwrites in its new order
    lp_status r = rebuild_decision(c, cin, c->cfg.skin > 0.0 ? 0 : 1, first);
    if (r == LP_OK) r = cells_build_device(c, in, ids, c->w.gate, bits);
    if (r == LP_OK) r = tile_map_build(c, c->w.gate);
    const double* sorted[7];
    for (int a = 0; a < 7; ++a) sorted[a] = c->w.sst[a];
    if (r == LP_OK) r = stencils_build(c, sorted, true);
    if (r == LP_OK) r = step_rhs(c, sorted);
    if (r == LP_OK) r = step_update(c, sorted, dt, in);
    return r;
}

}  // namespace
}  // namespace lp

using namespace lp;

extern "C" {

void lp_config_default(lp_config* cfg)
{
    if (!cfg) return;
    cfg->m_max = 60;
    cfg->precision = LP_FP64;
    cfg->cond_max = 20.0;
    cfg->weight = LP_W_UNIT;
    cfg->ghost_margin = 0.5;
    cfg->fallback_tol = 1e-12;
    cfg->debug_flags = 0;
    cfg->skin = 0.1;
    cfg->wall_reflect = 0;
    cfg->wall_pressure = 0;
    cfg->fit_order = 2;
    cfg->min_real_rows = 0;
}

lp_status lp_create(lp_ctx** out, void* stream, const lp_config* cfg)
{
    if (!out) return LP_E_ARG;
    *out = nullptr;
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
    lp_ctx* c = new (std::nothrow) lp_ctx();
    if (!c) return LP_E_ARG;
    c->stream = (hipStream_t)stream;
    c->cfg = c0;
    if (c0.debug_flags & LP_DEBUG_LANES2) c->lpp1 = c->lpp2 = 2;
    if (c0.debug_flags & LP_DEBUG_LANES4) c->lpp1 = c->lpp2 = 4;
    if (c0.debug_flags & LP_DEBUG_CLASSES) {
        // every class dispatch form: lanes 1, 4 and the staged tile kernel
        // in the first fit, 4, 2 and 1 in the second
        c->classes = true;
        const int l1[NCLASS] = {1, 4, 0}, l2[NCLASS] = {4, 2, 1};
        for (int k = 0; k < NCLASS; ++k) {
            c->cls_lpp1[k] = l1[k];
            c->cls_lpp2[k] = l2[k];
        }
    }
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LP_E_HIP;
    }
    *out = c;
    return LP_OK;
}

void lp_destroy(lp_ctx* c)
{
    if (!c) return;
    hipStreamSynchronize(c->stream);
    drop_graph(c);
    if (c->map_stream) {
        hipStreamSynchronize(c->map_stream);
        hipStreamDestroy(c->map_stream);
    }
    if (c->map_fork) hipEventDestroy(c->map_fork);
    if (c->map_join) hipEventDestroy(c->map_join);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    for (int q = 0; q < 16; ++q)
        if (c->ev[q]) hipEventDestroy(c->ev[q]);
    if (c->chk_ev) hipEventDestroy(c->chk_ev);
    free_work(c->w);
    delete c;
}

const char* lp_last_error(const lp_ctx* c)
{
    if (!c) return "null context";
    return c->err.c_str();
}

lp_status lp_reserve(lp_ctx* c, int64_t n_max, int64_t cells_max)
{
    if (c) drop_graph(c);
    if (!c || n_max < 1 || cells_max < 1 || n_max >= (1ll << 27)) {
        if (c) c->err = "lp_reserve: n_max in [1, 2^27), cells_max >= 1";
        return LP_E_ARG;
    }
    hipStreamSynchronize(c->stream);
    Work& w = c->w;
    free_work(w);
    const int64_t nb = (n_max + SORT_TILE - 1) / SORT_TILE;
    const int mm = c->cfg.m_max;
    hipError_t e = hipSuccess;
    work_layout(w, n_max, cells_max, mm, SYS_CAP, false, [&](auto*& p, int64_t cnt) {
        if (e == hipSuccess) e = alloc(p, cnt);
    });
    if (e == hipSuccess) e = hipHostMalloc((void**)&w.h_summary, sizeof(Summary));
    if (e == hipSuccess) e = hipMemset(w.err, 0, sizeof(ErrWord));
    if (e == hipSuccess) e = hipMemset(w.cnt, 0, sizeof(Counters));
    if (e == hipSuccess) e = hipMemset(w.summary, 0, sizeof(Summary));
    // no tile is staged until a neighbour list is built
    if (e == hipSuccess)
        e = hipMemset(w.tile_cnt, 0xFF, sizeof(int32_t) * ((n_max + BLOCK - 1) / BLOCK));
    if (e == hipSuccess) {
        ErrWord ew{0, 0, ~0ull};
        e = hipMemcpy(w.err, &ew, sizeof(ew), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_work(w);
        return hip_fail(c, e, "lp_reserve");
    }
    w.n_max = n_max;
    w.cells_max = cells_max;
    w.m_max = mm;
    w.hist_cap = RADIX_MAX_DIGITS * nb;
    c->cells_ok = c->stencils_ok = c->list_ok = c->map_ok = false;
    c->redo_clear = c->disp_clear = false;
    if (c->n_sys > 0) {
        // re-upload the systems into the new buffers
        std::vector<int64_t> off = c->h_off;
        std::vector<lp_params> prm = c->h_prm;
        return lp_set_systems(c, c->n_sys, off.data(), prm.data());
    }
    return LP_OK;
}

lp_status lp_set_systems(lp_ctx* c, int32_t n_sys, const int64_t* offsets,
                         const lp_params* params)
{
    if (!c) return LP_E_ARG;
    if (n_sys < 1 || n_sys > SYS_CAP || !offsets || !params) {
        c->err = "lp_set_systems: 1 <= n_sys <= 4096 with host offsets and params";
        return LP_E_ARG;
    }
    if (offsets[0] != 0) {
        c->err = "offsets[0] must be 0";
        return LP_E_ARG;
    }
    for (int s = 0; s < n_sys; ++s) {
        if (offsets[s + 1] < offsets[s]) {
            c->err = "offsets must be non-decreasing";
            return LP_E_ARG;
        }
        const lp_params& p = params[s];
        const bool ok = p.phi_min < p.phi_max && p.phi_max < p.phi_c &&
                        p.phi_min > 0.0 && p.beta > 0.0 && p.R > 0.0 &&
                        p.h > 0.0 && p.rho_s > 0.0 && p.d > 0.0 && p.I0 > 0.0 &&
                        std::isfinite(p.wall_z) && std::isfinite(p.alpha) &&
                        std::isfinite(p.g[0]) && std::isfinite(p.g[1]) &&
                        std::isfinite(p.g[2]) && std::isfinite(p.mu_s) &&
                        std::isfinite(p.mu_2);
        if (!ok) {
            c->err = "invalid parameters of system " + std::to_string(s);
            return LP_E_ARG;
        }
        // a periodic axis holds at least three list cells, so that each
        // pair in the list has one nearest copy
        const double cmin = p.R * (1.0 + c->cfg.skin) * (1.0 + 1.0 / 1048576.0);
        for (int a = 0; a < 2; ++a) {
            const double L = p.box_len[a];
            if (!(L >= 0.0) || !std::isfinite(L) || !std::isfinite(p.box_lo[a]) ||
                (L > 0.0 && !(L >= 3.0 * cmin))) {
                c->err = "system " + std::to_string(s) +
                         ": a periodic period must be 0 (open) or at least "
                         "3 R (1 + skin)";
                return LP_E_ARG;
            }
        }
    }
    if (offsets[n_sys] >= (1ll << 27)) {
        c->err = "at most 2^27 - 1 particles";
        return LP_E_ARG;
    }
    c->h_off.assign(offsets, offsets + n_sys + 1);
    c->h_prm.assign(params, params + n_sys);
    c->periodic = false;
    for (const lp_params& p : c->h_prm)
        if (p.box_len[0] > 0.0 || p.box_len[1] > 0.0) c->periodic = true;
    c->n_sys = n_sys;
    c->n = offsets[n_sys];
    c->cells_ok = c->stencils_ok = c->list_ok = c->map_ok = false;
    if (c->w.n_max == 0) return LP_OK;   // uploaded by lp_reserve
    hipError_t e = hipMemcpyAsync(c->w.off, c->h_off.data(),
                                  sizeof(int64_t) * (n_sys + 1),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->w.prm, c->h_prm.data(), sizeof(lp_params) * n_sys,
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "lp_set_systems upload");
    return LP_OK;
}

lp_status lp_build_cells(lp_ctx* c, lp_state* s, int32_t* perm)
{
    if (!s) return LP_E_ARG;
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    double* st[7];
    state_arrays(s, st);
    r = cells_build(c, st, perm);
    if (r == LP_OK) r = state_write_back(c, st);
    if (r == LP_OK) c->built_x = s->x;
    return r;
}

lp_status lp_neighbors(lp_ctx* c, const lp_state* s, int64_t* cand_off,
                       int32_t* cand_idx, int64_t cap, int64_t* needed,
                       int32_t* sten_cnt, int32_t* sten_idx,
                       uint8_t* ghost_mask, int64_t* n_mirror)
{
    if (!s) return LP_E_ARG;
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    if (!c->cells_ok || !c->list_ok || c->built_x != s->x) {
        c->err = "lp_build_cells must be called on this state first";
        return LP_E_STATE;
    }
    double* st[7];
    state_arrays(s, st);
    r = stencils_build(c, st);
    if (r != LP_OK) return r;
    return stencils_export(c, st, cand_off, cand_idx, cap, needed, sten_cnt,
                           sten_idx, ghost_mask, n_mirror);
}

lp_status lp_fit_derivs(lp_ctx* c, const lp_state* s, const double* f,
                        int32_t k, const int32_t* mirror_sign,
                        const int32_t* ghost_zero, double* coef,
                        uint8_t* flags)
{
    if (!s || !f || !coef || !mirror_sign || !ghost_zero || k < 1 || k > 8) {
        if (c) c->err = "lp_fit_derivs: 1 <= k <= 8 and non-null arrays";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    if (!c->stencils_ok || c->built_x != s->x) {
        c->err = "lp_neighbors must be called on this state first";
        return LP_E_STATE;
    }
    double* st[7];
    state_arrays(s, st);
    return fit_generic(c, st, f, k, mirror_sign, ghost_zero, coef, flags);
}

lp_status lp_rheology_rhs(lp_ctx* c, const lp_state* s, const double* coef_u,
                          double* dVdt, double* acc, double* diag, double* grad,
                          uint8_t* flags)
{
    if (!s || !coef_u || !dVdt || !acc) {
        if (c) c->err = "lp_rheology_rhs: coef_u, dVdt and acc are required";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    if (!c->stencils_ok || c->built_x != s->x) {
        c->err = "lp_neighbors must be called on this state first";
        return LP_E_STATE;
    }
    double* st[7];
    state_arrays(s, st);
    return rhs_from_coef(c, st, coef_u, dVdt, acc, diag, grad, flags);
}

// The displacement check of a step on the current list, with the state
// copied into the working state: its result comes back to the host while
// the stream already runs the mirrors and the histogram selection on the
// current list (when its tile map is current), which a rebuild then
// repeats.  rebuild: some particle moved `limit` skins or more; ahead: the
// selection was enqueued (the step then adds only its tail).
static lp_status check_ahead(lp_ctx* c, double* const in[7], const double* const sorted[7],
                             double limit, bool* rebuild, bool* ahead)
{
    lp_status r = list_check_start(c, in);
    if (r != LP_OK) return r;
    *ahead = c->chk_pending && c->map_ok;
    if (*ahead) {
        prof_mark(c, 0, true);
        r = stencils_build(c, sorted, true, STENCIL_HEAD);
        if (r != LP_OK) return r;
    }
    double ratio = -1.0;
    r = list_check_wait(c, &ratio);
    if (r != LP_OK) return r;
    *rebuild = !(ratio >= 0.0) || !(std::sqrt(ratio) < limit);
    return LP_OK;
}

// The tile map of a list just built, on the side stream after the list
// (fork); tile_map_join makes the step's stream wait for it.
static lp_status tile_map_fork(lp_ctx* c)
{
    hipError_t e = hipSuccess;
    if (!c->map_stream) e = hipStreamCreateWithFlags(&c->map_stream, hipStreamNonBlocking);
    if (e == hipSuccess && !c->map_fork)
        e = hipEventCreateWithFlags(&c->map_fork, hipEventDisableTiming);
    if (e == hipSuccess && !c->map_join)
        e = hipEventCreateWithFlags(&c->map_join, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(c->map_fork, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->map_stream, c->map_fork, 0);
    if (e != hipSuccess) return hip_fail(c, e, "tile map fork");
    hipStream_t own = c->stream;
    c->stream = c->map_stream;
    lp_status r = tile_map_build(c);
    c->stream = own;
    if (r != LP_OK) return r;
    e = hipEventRecord(c->map_join, c->map_stream);
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "tile map join");
}

static lp_status tile_map_join(lp_ctx* c)
{
    const hipError_t e = hipStreamWaitEvent(c->stream, c->map_join, 0);
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "tile map join");
}

lp_status lp_step(lp_ctx* c, lp_state* s, double dt, int32_t* perm,
                  lp_step_record* rec)
{
    if (!s || !(dt > 0.0) || !std::isfinite(dt)) {
        if (c) c->err = "lp_step: dt must be positive and finite";
        return LP_E_ARG;
    }
    if (rec && !rec->perm) {
        if (c) c->err = "lp_step: a step record needs its perm array";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    double* in[7];
    state_arrays(s, in);
    prof_mark(c, 0, false);
    const double* sorted[7];
    double* const* sst = c->w.sst;
    for (int a = 0; a < 7; ++a) sorted[a] = sst[a];
    // the neighbour list stays valid until some particle has moved half
    // the skin since the last build
    bool rebuild = !c->list_ok || !(c->cfg.skin > 0.0) || (rec && rec->force_sort);
    bool ahead = false;
    if (!rebuild) {
        r = check_ahead(c, in, sorted, 0.49, &rebuild, &ahead);
        if (r != LP_OK) return r;
    }
    if (rebuild) {
        r = cells_build(c, in, rec ? rec->perm : perm);
        if (r == LP_OK && rec && perm) r = copy_perm(c, rec->perm, perm);
    } else {
        r = state_copy(c, in, perm, nullptr, false);
    }
    bool forked = false;
    if (r == LP_OK && !c->map_ok && c->map_side) {
        r = tile_map_fork(c);
        forked = r == LP_OK;
    } else if (r == LP_OK && !c->map_ok) {
        r = tile_map_build(c);
    }
    if (!ahead || rebuild) prof_mark(c, 0, true);
    if (r != LP_OK) return r;
    if (rebuild) ++c->rebuilds;
    if (rec) {
        rec->resorted = rebuild ? 1 : 0;
        rec->list_gen = c->list_gen;
    }
    // the displacement check's copy or the re-sort packed the positions
    r = stencils_build(c, sorted, true, ahead && !rebuild ? STENCIL_TAIL : STENCIL_ALL);
    if (r == LP_OK && forked) r = tile_map_join(c);
    if (r == LP_OK) r = step_rhs(c, sorted);
    if (r == LP_OK) r = step_update(c, sorted, dt, in);
    // stencils of the API calls refer to lp_build_cells' state
    c->stencils_ok = false;
    c->built_x = nullptr;
    if (r == LP_OK && c->prof) {
        hipError_t e = hipEventSynchronize(c->ev[13]);
        if (e != hipSuccess) return hip_fail(c, e, "profile sync");
        for (int ph = 0; ph < 7; ++ph) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev[2 * ph], c->ev[2 * ph + 1]) == hipSuccess)
                c->prof_ms[ph] += ms;
        }
        ++c->prof_steps;
    }
    return r;
}

lp_status lp_step2(lp_ctx* c, lp_state* s, double dt, int32_t* perm,
                   lp_step_record* rec)
{
    if (!s || !(dt > 0.0) || !std::isfinite(dt)) {
        if (c) c->err = "lp_step2: dt must be positive and finite";
        return LP_E_ARG;
    }
    if (rec && !rec->perm) {
        if (c) c->err = "lp_step2: a step record needs its perm array";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    if (!(c->cfg.skin > 0.0)) {
        c->err = "lp_step2 needs a neighbour-list skin > 0 (its predictor stage "
                 "reuses the list)";
        return LP_E_ARG;
    }
    double* in[7];
    state_arrays(s, in);
    const double* sorted[7];
    for (int a = 0; a < 7; ++a) sorted[a] = c->w.sst[a];
    // rebuild earlier than lp_step: the predictor stage moves particles a
    // further dt |u| on the same list and must stay within half the skin
    bool rebuild = !c->list_ok || (rec && rec->force_sort);
    bool ahead = false;
    if (!rebuild) {
        r = check_ahead(c, in, sorted, 0.4, &rebuild, &ahead);
        if (r != LP_OK) return r;
    }
    if (rebuild) {
        r = cells_build(c, in, rec ? rec->perm : perm);
        if (r == LP_OK && rec && perm) r = copy_perm(c, rec->perm, perm);
    } else {
        r = state_copy(c, in, perm, nullptr, false);
    }
    if (r == LP_OK && !c->map_ok) r = tile_map_build(c);
    if (r != LP_OK) return r;
    if (rebuild) ++c->rebuilds;
    if (rec) {
        rec->resorted = rebuild ? 1 : 0;
        rec->list_gen = c->list_gen;
    }
    r = stencils_build(c, sorted, true, ahead && !rebuild ? STENCIL_TAIL : STENCIL_ALL);
    if (r == LP_OK) r = step_rhs(c, sorted);
    if (r == LP_OK) r = step_pass2(c, sorted, dt, nullptr, c->w.acc, c->w.dVdt);
    if (r == LP_OK) r = step_heun(c, dt, in);
    c->stencils_ok = false;
    c->built_x = nullptr;
    return r;
}

lp_status lp_profile(lp_ctx* c, int32_t enable)
{
    if (!c) return LP_E_ARG;
    if (enable && !c->ev[0])
        for (int q = 0; q < 16; ++q) {
            hipError_t e = hipEventCreate(&c->ev[q]);
            if (e != hipSuccess) return hip_fail(c, e, "lp_profile");
        }
    c->prof = enable != 0;
    return LP_OK;
}

lp_status lp_profile_read(lp_ctx* c, double* ms8, int64_t* steps)
{
    if (!c || !ms8) return LP_E_ARG;
    for (int q = 0; q < 8; ++q) {
        ms8[q] = c->prof_ms[q];
        c->prof_ms[q] = 0.0;
    }
    if (steps) *steps = c->prof_steps;
    c->prof_steps = 0;
    return LP_OK;
}

lp_status lp_autotune(lp_ctx* c, const lp_state* s, int32_t* choice)
{
    if (!s) {
        if (c) c->err = "lp_autotune: null state";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    double* in[7];
    state_arrays(s, in);
    r = cells_build(c, in, nullptr);
    // with the tile map, as the steps run the fits
    if (r == LP_OK) r = tile_map_build(c);
    const double* sorted[7];
    for (int a = 0; a < 7; ++a) sorted[a] = c->w.sst[a];
    if (r == LP_OK) r = stencils_build(c, sorted);
    if (r == LP_OK) r = autotune_fits(c, sorted, choice);
    // the working copy is a sorted copy of s, not the caller's order
    c->list_ok = false;
    c->stencils_ok = false;
    c->built_x = nullptr;
    drop_graph(c);
    return r;
}

lp_status lp_fit_plan(lp_ctx* c, int32_t* plan, double* ms)
{
    if (!c || !plan) return LP_E_ARG;
    plan[0] = c->lpp1;
    plan[1] = c->lpp2;
    plan[2] = (c->classes && c->cfg.fit_order == 2 && c->cfg.precision == LP_FP64) ? 1 : 0;
    for (int k = 0; k < NCLASS; ++k) {
        plan[3 + k] = c->cls_lpp1[k];
        plan[6 + k] = c->cls_lpp2[k];
        plan[9 + k] = (int32_t)c->cls_count[k];
    }
    if (ms)
        for (int q = 0; q < 8; ++q) ms[q] = c->tune_ms[q];
    return LP_OK;
}

lp_status lp_step_graph(lp_ctx* c, lp_state* s, int32_t* ids, double dt,
                        int32_t nsteps)
{
    if (!s || !(dt > 0.0) || !std::isfinite(dt) || nsteps < 1 || nsteps > 4096) {
        if (c) c->err = "lp_step_graph: dt > 0 and 1 <= nsteps <= 4096";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    double* in[7];
    state_arrays(s, in);
    Work& w = c->w;
    if (!c->list_ok) {
        // first build, eagerly, into the caller's arrays (as lp_build_cells)
        r = cells_build(c, in, w.adj_perm);
        if (r == LP_OK) r = state_write_back(c, in);
        if (r == LP_OK && ids) r = permute_ids(c, w.adj_perm, ids);
        if (r != LP_OK) return r;
    }
    // the captured steps keep list and tile map together; a list built
    // since by another entry point gets its map here
    if (!c->map_ok) {
        r = tile_map_build(c);
        if (r != LP_OK) return r;
    }
    const int bits = std::min(16, c->axis_bits + 1);
    lp_ctx::GraphKey key{};
    for (int a = 0; a < 7; ++a) key.st[a] = in[a];
    key.ids = ids;
    key.dt = dt;
    key.nsteps = nsteps;
    key.bits = bits;
    key.n = c->n;
    key.n_sys = c->n_sys;
    if (!c->gexec || !(key == c->gkey)) {
        drop_graph(c);
        hipError_t e = hipSuccess;
        if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(c, e, "capture stream");
        hipStream_t saved = c->stream;
        const bool prof = c->prof;
        c->prof = false;
        c->stream = c->cap_stream;
        e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            c->stream = saved;
            c->prof = prof;
            return hip_fail(c, e, "begin capture");
        }
        for (int k = 0; k < nsteps && r == LP_OK; ++k)
            r = step_device(c, in, ids, dt, bits, k == 0);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->cap_stream, &g);
        c->stream = saved;
        c->prof = prof;
        // what the captured kernels leave is not tracked on the host
        c->redo_clear = c->disp_clear = false;
        if (r != LP_OK) {
            if (g) hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return hip_fail(c, e, "end capture");
        c->graph = g;
        e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            drop_graph(c);
            return hip_fail(c, e, "graph instantiate");
        }
        c->gkey = key;
    }
    hipError_t e = hipGraphLaunch(c->gexec, c->stream);
    c->redo_clear = c->disp_clear = false;
    if (e != hipSuccess) return hip_fail(c, e, "graph launch");
    // the replay may have rebuilt the list on the device: records of
    // earlier steps no longer describe the current list
    ++c->list_gen;
    c->stencils_ok = false;
    c->built_x = nullptr;
    return LP_OK;
}

lp_status lp_step_adjoint(lp_ctx* c, const lp_state* s, double dt,
                          const lp_state* adj_out, lp_state* adj_in,
                          double* adj_params, int32_t* perm,
                          const lp_step_record* rec)
{
    if (!s || !adj_out || !adj_in || !adj_params || !(dt > 0.0) || !std::isfinite(dt)) {
        if (c) c->err = "lp_step_adjoint: null argument or dt not positive";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    if (c->cfg.weight != LP_W_UNIT || c->cfg.wall_reflect || c->cfg.wall_pressure ||
        c->cfg.fit_order != 2) {
        c->err = "lp_step_adjoint supports unit weights, quadratic fits and the "
                 "mirror wall only";
        return LP_E_ARG;
    }
    double* in[7];
    state_arrays(s, in);
    const int32_t* order = nullptr;
    r = adjoint_order(c, in, rec, &order);
    const double* sorted[7];
    for (int a = 0; a < 7; ++a) sorted[a] = c->w.sst[a];
    // (the working copy came with its positions' records)
    if (r == LP_OK) r = stencils_build(c, sorted, true);
    if (r == LP_OK) r = step_pass1_coef(c, sorted);
    double* lam_in[7];
    double* out[7];
    state_arrays(adj_out, lam_in);
    state_arrays(adj_in, out);
    AdjSeed seed;
    for (int a = 0; a < 7; ++a) seed.A[a] = lam_in[a];
    seed.c_ux = seed.c_a = seed.c_d = dt;
    seed.k_x = 0.5 * dt;
    if (r == LP_OK) r = step_adjoint(c, sorted, seed, out, adj_params, order);
    if (r == LP_OK && perm) r = order ? copy_perm(c, order, perm)
                                      : state_copy(c, nullptr, perm, nullptr, false);
    // without a record the list was built for this call: the next lp_step
    // rebuilds
    if (!rec) c->list_ok = false;
    c->stencils_ok = false;
    c->built_x = nullptr;
    return r;
}

lp_status lp_step2_adjoint(lp_ctx* c, const lp_state* s, double dt,
                           const lp_state* adj_out, lp_state* adj_in,
                           double* adj_params, int32_t* perm,
                           const lp_step_record* rec)
{
    if (!s || !adj_out || !adj_in || !adj_params || !(dt > 0.0) || !std::isfinite(dt)) {
        if (c) c->err = "lp_step2_adjoint: null argument or dt not positive";
        return LP_E_ARG;
    }
    lp_status r = check_ready(c, s);
    if (r != LP_OK) return r;
    if (c->cfg.weight != LP_W_UNIT || c->cfg.wall_reflect || c->cfg.wall_pressure ||
        c->cfg.fit_order != 2) {
        c->err = "lp_step2_adjoint supports unit weights, quadratic fits and the "
                 "mirror wall only";
        return LP_E_ARG;
    }
    if (!(c->cfg.skin > 0.0)) {
        c->err = "lp_step2_adjoint needs a neighbour-list skin > 0";
        return LP_E_ARG;
    }
    Work& w = c->w;
    double* in[7];
    state_arrays(s, in);
    double* lam_in[7];
    double* out[7];
    state_arrays(adj_out, lam_in);
    state_arrays(adj_in, out);
    const double* sorted[7];
    const double* pred[7];
    for (int a = 0; a < 7; ++a) {
        sorted[a] = w.sst[a];
        pred[a] = w.sst2[a];
    }
    // forward: s (in the step's order), f(s) in float64, predictor s*, its
    // stencils
    const int32_t* order = nullptr;
    r = adjoint_order(c, in, rec, &order);
    if (r == LP_OK) r = stencils_build(c, sorted, true);
    if (r == LP_OK) r = step_pass1_coef(c, sorted);
    if (r == LP_OK) r = step_pass2(c, sorted, 0.0, nullptr, w.acc, w.dVdt, true);
    if (r == LP_OK) r = heun_predictor(c, dt);
    if (r == LP_OK) r = stencils_build(c, pred);
    if (r == LP_OK) r = step_pass1_coef(c, pred);
    // corrector stage: s' = s + dt/2 (f(s) + f(s*)) seen from s*: its
    // cotangent lam* = J_f(s*)^T (dt/2 lam') lands in adj2
    AdjSeed s2;
    for (int a = 0; a < 7; ++a) s2.A[a] = lam_in[a];
    s2.iA = 0.0;
    s2.c_ux = s2.c_a = s2.c_d = 0.5 * dt;
    if (r == LP_OK) r = step_adjoint(c, pred, s2, w.adj2, adj_params, nullptr);
    // predictor stage seen from s: identity lam' + lam*, and f(s) with
    // cotangent dt (lam'/2 + lam*)
    if (r == LP_OK) r = stencils_build(c, sorted);
    if (r == LP_OK) r = step_pass1_coef(c, sorted);
    AdjSeed s1;
    for (int a = 0; a < 7; ++a) {
        s1.A[a] = lam_in[a];
        s1.B[a] = w.adj2[a];
    }
    s1.iA = s1.iB = 1.0;
    s1.nA = 0.5;
    s1.nB = 1.0;
    s1.c_ux = s1.c_a = s1.c_d = dt;
    if (r == LP_OK) r = step_adjoint(c, sorted, s1, out, adj_params, order);
    if (r == LP_OK && perm) r = order ? copy_perm(c, order, perm)
                                      : state_copy(c, nullptr, perm, nullptr, false);
    if (!rec) c->list_ok = false;
    c->stencils_ok = false;
    c->built_x = nullptr;
    return r;
}

lp_status lp_sync_status(lp_ctx* c, int64_t* index)
{
    if (!c) return LP_E_ARG;
    if (index) *index = -1;
    if (!c->w.err) return LP_OK;
    ErrWord ew;
    hipError_t e = hipMemcpyAsync(&ew, c->w.err, sizeof(ew), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "lp_sync_status");
    if (ew.code == 0) return LP_OK;
    ErrWord clear{0, 0, ~0ull};
    e = hipMemcpyAsync(c->w.err, &clear, sizeof(clear), hipMemcpyHostToDevice,
                       c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (index) *index = (int64_t)ew.index;
    if (ew.code & ERR_BOX) {
        c->err = "particle " + std::to_string(ew.index) +
                 " lies more than one period outside its periodic box";
        return LP_E_ARG;
    }
    if (ew.code & ERR_LIST) {
        c->err = "the predictor stage of a second-order step moved particle " +
                 std::to_string(ew.index) +
                 " beyond the neighbour-list skin: reduce dt or increase skin";
        return LP_E_STATE;
    }
    if (ew.code & ERR_CAPACITY) {
        c->err = "device capacity exceeded (too many candidates for the sorted "
                 "stencil path) at particle " + std::to_string(ew.index);
        return LP_E_CAPACITY;
    }
    c->err = "non-finite state at particle " + std::to_string(ew.index);
    return LP_E_NUMERIC;
}

lp_status lp_stats(lp_ctx* c, int64_t* out8)
{
    if (!c || !out8) return LP_E_ARG;
    for (int q = 0; q < 8; ++q) out8[q] = 0;
    out8[0] = c->n;
    if (!c->w.cnt) return LP_OK;
    Counters k;
    int64_t nm = 0;
    hipError_t e = hipMemcpyAsync(&k, c->w.cnt, sizeof(k), hipMemcpyDeviceToHost,
                                  c->stream);
    // mirrors of the last stencil build
    if (e == hipSuccess)
        e = hipMemcpyAsync(&nm, &c->w.summary->n_mirror, sizeof(nm),
                           hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    out8[1] = nm;
    if (e != hipSuccess) return hip_fail(c, e, "lp_stats");
    out8[2] = (int64_t)k.qr_refits;
    out8[3] = (int64_t)k.hard_stencils;
    out8[4] = (int64_t)k.below_wall;
    out8[5] = c->rebuilds + (int64_t)k.rebuilds;
    c->rebuilds = 0;
    // tiles of the current neighbour list, and those the fits cannot stage
    if (c->list_ok && c->n > 0 && !c->map_ok) {
        // no tile map for this list: the fits read every neighbour globally
        out8[6] = out8[7] = (c->n + BLOCK - 1) / BLOCK;
    } else if (c->list_ok && c->n > 0) {
        const int64_t tiles = (c->n + BLOCK - 1) / BLOCK;
        std::vector<int32_t> tc((size_t)tiles);
        e = hipMemcpy(tc.data(), c->w.tile_cnt, sizeof(int32_t) * tiles,
                      hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(c, e, "lp_stats");
        int64_t off = 0;
        for (int32_t v : tc) off += (v < 0 || v > STAGE_CAP) ? 1 : 0;
        out8[6] = off;
        out8[7] = tiles;
    }
    Counters z{};
    e = hipMemcpyAsync(c->w.cnt, &z, sizeof(z), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? LP_OK : hip_fail(c, e, "lp_stats reset");
}

}  // extern "C"
