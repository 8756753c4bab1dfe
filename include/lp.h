/*
 * lp.h — C ABI of the MI355X (gfx950) library for one explicit time step
 * of the Lagrangian-particle (LP) method for granular flow with mu(I)
 * rheology (Zepeda & Samulyak, arXiv:2206.14061).
 *
 * The step (Sec. 3.1 of the paper, steps 5-10) is:
 *   mirrors for the solid wall (step 9) -> neighbour search (step 5) ->
 *   stencils with octant coverage and ghost completion (steps 5-6) ->
 *   second-order least-squares derivatives (step 7) -> mu(I) closure
 *   (Sec. 2.2, 2.2.1) -> second fit of P and eta -> momentum and volume
 *   right-hand side (Sec. 2.1) -> explicit update (steps 8 and 10).
 * The paper's octree (step 4) is replaced by a Morton-sorted uniform cell
 * list (lp_build_cells).
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers owned by the caller unless marked
 *    "host".  All floating point is IEEE float64.  Particle ids are int32
 *    (at most 2^28 - 1 real + mirror particles).
 *  - Work is enqueued asynchronously on the stream given to lp_create.
 *    Only calls that return host values (lp_build_cells, lp_neighbors'
 *    counts, lp_sync_status) synchronise that stream.  An lp_step that
 *    builds a new neighbour list runs one kernel on a second stream of the
 *    library's (default priority), forked from and joined back into that
 *    stream within the call, so work ordered after the call on that stream
 *    sees all of it.
 *  - Every call returns an lp_status; nothing throws across the ABI.
 *    lp_last_error() gives a text description of the last failure.
 *    Failures detected on the device (capacity overflow, non-finite
 *    results) are latched in a device error word and reported by
 *    lp_sync_status().
 *  - After lp_reserve() no call allocates device memory.
 *  - Particles of system s occupy the index range [offsets[s],
 *    offsets[s+1]) and never interact with other systems.
 *  - A context is not thread safe; calls that overlap on one context race.
 */
#ifndef LP_H
#define LP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LP_OK = 0,
    LP_E_ARG = 1,       /* invalid argument (null, size, parameter range)   */
    LP_E_CAPACITY = 2,  /* workspace or output capacity exceeded            */
    LP_E_NUMERIC = 3,   /* non-finite state produced                        */
    LP_E_HIP = 4,       /* HIP runtime error                                */
    LP_E_STATE = 5      /* call order violated or entry point unavailable   */
} lp_status;

enum { LP_FP64 = 0, LP_FP32_REFINED = 1 };
enum { LP_W_UNIT = 0, LP_W_GAUSS = 1 };

/* debug_flags: route every particle through the exact slow paths, fix
 * the lanes per particle of the fits (see lp_autotune), make the fits
 * read every neighbour from global memory instead of from the tile's
 * neighbours staged in LDS, or dispatch the fits by stencil size class
 * (classes of at most 16, at most 32 and more rows; lanes per particle 1,
 * 4 and the staged tile kernel in the first fit, 4, 2 and 1 in the
 * second; results agree to rounding), number mirrors through a separate
 * scan of the tile counts, or build the neighbour list with a thread per
 * particle instead of a wavefront per cell (the lists are identical) */
enum { LP_DEBUG_SORTED_STENCIL = 1, LP_DEBUG_QR_FIT = 2, LP_DEBUG_LANES2 = 4,
       LP_DEBUG_LANES4 = 8, LP_DEBUG_GLOBAL_GATHER = 16, LP_DEBUG_CLASSES = 32,
       LP_DEBUG_MIRROR_SCAN = 64, LP_DEBUG_PARTICLE_LIST = 128 };

/* Physical constants of one system (Sec. 2.2, 2.2.1 and Sec. 4).
 * rho_s: grain material density (the paper's phi_s); d: grain diameter;
 * mu_s, mu_2, I0: friction law mu(I) = mu_s + (mu_2 - mu_s)/(I0/I + 1);
 * phi_c, phi_min: critical and minimum solid fraction (eq.
 * inertialdensity, a = phi_c - phi_min); phi_max: start of the
 * quasi-static branch; alpha, beta: quasi-static pressure
 * P = rho_s (alpha + beta phi) (eq. CST2); g: body force; h: particle
 * spacing (fit scaling, ghost offset); R: neighbour radius; wall_z: solid
 * wall plane z = wall_z (mirror boundary).  box_lo, box_len: periodic
 * boundary (Sec. 3.1, boundary conditions) along x (index 0) and y
 * (index 1): an axis with box_len > 0 identifies x with x + box_len;
 * particles see the copy of each neighbour nearest to them (x_j - L when
 * x_j - x_i > L/2, x_j + L when below -L/2), and the steps map positions
 * back into [box_lo, box_lo + box_len).  box_len = 0 leaves the axis open.
 * Requires phi_min < phi_max < phi_c, beta > 0, R > 0, h > 0, and on a
 * periodic axis box_len >= 3 R (1 + skin) (1 + 2^-20) with positions
 * within one period of the box. */
typedef struct {
    double rho_s, d, mu_s, mu_2, I0, phi_c, phi_min, phi_max, alpha, beta;
    double g[3];
    double h, R, wall_z;
    double box_lo[2], box_len[2];
} lp_params;

/* Numerical configuration of a context.
 * m_max: stencil cap (1..64; default 60).  precision: LP_FP64 or
 * LP_FP32_REFINED.  cond_max (default 20): a stencil whose Cholesky pivot
 * ratio min U_jj / max U_jj of the Gram matrix falls below 1/cond_max (4
 * times that in refined FP32) is refitted by FP64 Householder QR; at 20
 * this keeps cond(G) below about 1e5 on the tested stencils, so the
 * normal equations stay within 1e-10 of QR.  weight: LP_W_UNIT or
 * LP_W_GAUSS (w = exp(-4 r^2 / R^2)).  ghost_margin: an octant is covered
 * when a neighbour lies beyond ghost_margin * h on every axis (0.5).
 * fallback_tol: stencils with min|r_jj|/max|r_jj| below it (or fewer than 9
 * rows) use a linear fit (1e-12).  debug_flags: LP_DEBUG_* bits (sorted
 * stencil path for every particle, Householder refit for every stencil,
 * 2 or 4 lanes per particle in the fits, mirror numbering through a
 * separate scan of the per-tile counts as above 2048 tiles of 4,096
 * particles).
 * skin: neighbour-list margin in units of R (default 0.1): the list holds
 * every pair within R (1 + skin) and is rebuilt (with a Morton re-sort)
 * once a particle has moved skin R / 2 since the last build; 0 rebuilds
 * at every step.  Results do not depend on it except through the particle
 * order (ids), which changes only at rebuilds.
 * wall_reflect (default 0): with 1, a step that leaves a particle below the
 * wall plane reflects it across the plane (z -> 2 wall_z - z, w -> -w);
 * the paper states only the mirror boundary, through which particles can
 * sink when the mirror pressure under-supports them.
 * wall_pressure (default 0): with 1, a mirror's pressure (Sec. 3.1 step 9:
 * P(phi_src) at zero shear rate) gains the hydrostatic weight of the layer
 * between mirror and source, rho_s phi_src |g_z| (z_src - z_mirror)
 * (the generalized wall condition of Adami, Hu & Adams, J. Comput. Phys.
 * 231 (2012)); with the literal mirror a column at rest carries only about
 * a third of its bottom row's weight.  The adjoint entry points require
 * both options at 0.
 * fit_order (default 2): 3 selects cubic fits (19 unknowns: the Taylor row
 * of Sec. 3.1 step 7 extended by the third-order terms, the higher-order
 * fit the paper lists as further work) in every fit; they fall back to the
 * quadratic fit below 19 rows or when min|r_jj|/max|r_jj| < fallback_tol
 * (flag bit 4), then to the linear one.  Cubic fits run in float64 with
 * one wavefront per particle whatever the precision setting, need
 * m_max <= 56 (stencil plus ghost rows fit one wavefront), and are not
 * available to the adjoint entry points.
 * min_real_rows (default 0, off): a stencil with fewer real or mirror
 * rows than this (ghost rows not counted) takes the linear fit (flag bit
 * 0) instead of the quadratic or cubic one; 9 (as many real rows as the
 * quadratic fit has unknowns) keeps a free-surface particle with a few
 * neighbours and many ghost rows from an interpolating quadratic fit. */
typedef struct {
    int32_t m_max;
    int32_t precision;
    double cond_max;
    int32_t weight;
    double ghost_margin;
    double fallback_tol;
    int32_t debug_flags;
    double skin;
    int32_t wall_reflect;
    int32_t wall_pressure;
    int32_t fit_order;
    int32_t min_real_rows;
} lp_config;

/* Structure-of-arrays particle state, device float64 arrays of length n
 * (total particles of all systems): position x y z, velocity u v w and
 * specific volume V = 1/phi. */
typedef struct {
    double *x, *y, *z, *u, *v, *w, *V;
} lp_state;

typedef struct lp_ctx lp_ctx;

/* Fills *cfg with the defaults listed above. */
void lp_config_default(lp_config* cfg);

/* Creates a context bound to the current HIP device and to `stream` (a
 * hipStream_t, may be null for the default stream).  cfg may be null for
 * the defaults.  *out receives the context. */
lp_status lp_create(lp_ctx** out, void* stream, const lp_config* cfg);

/* Releases the context and its workspace (null is ignored). */
void lp_destroy(lp_ctx* ctx);

/* Text of the last error on this context (never null). */
const char* lp_last_error(const lp_ctx* ctx);

/* Reserves workspace for up to n_max particles (mirrors included) and
 * cells_max cells per call.  Allocates; every later call on this context
 * allocates nothing.  May be called again to grow. */
lp_status lp_reserve(lp_ctx* ctx, int64_t n_max, int64_t cells_max);

/* Sets the systems: n_sys >= 1, offsets (host, n_sys + 1 entries,
 * offsets[0] = 0, non-decreasing), params (host, n_sys records).  Copies
 * both; validates parameter ranges (LP_E_ARG). */
lp_status lp_set_systems(lp_ctx* ctx, int32_t n_sys, const int64_t* offsets,
                         const lp_params* params);

/* Morton-sorted cell list and neighbour list (replace the octree of Sec.
 * 3.1 step 4 and Sec. 3.2).  Per system: origin (min x, min y,
 * min(min z, wall_z - R)), cell edge c = R (1 + skin) (1 + 2^-20), cell
 * coordinate floor((x - origin)/c), key = bit interleave of the cell
 * coordinates (x -> bit 3k, y -> 3k+1, z -> 3k+2).  Particles are
 * reordered in place by (system, key, old index); perm (device
 * int32[n], optional) receives perm[new] = old.  Then records for every
 * particle the reals within R (1 + skin) and the potential mirror sources
 * (Sec. 3.1 step 9: a mirror of every particle with z - wall_z < R, at
 * (x, y, 2 wall_z - z), velocity (u, v, -w), same V, id n + k in
 * ascending source order).  Synchronises the stream once (grid sizes).
 * LP_E_CAPACITY if the cells exceed the reservation or a cell coordinate
 * needs more than 16 bits; more than 256 list entries for a particle
 * latch LP_E_CAPACITY (lp_sync_status). */
lp_status lp_build_cells(lp_ctx* ctx, lp_state* s, int32_t* perm);

/* Neighbours, stencils and ghosts (Sec. 3.1 steps 5-6, free boundary of
 * step 9) of every real particle of the state passed to the last
 * lp_build_cells (positions changed since by less than skin R / 2):
 *  - candidates C_i = { j real or mirror of the same system, j != i :
 *    (dx*dx + dy*dy) + dz*dz < R*R in float64 without fused operations };
 *  - stencil: the nearest candidate (key (r^2, id)) of each octant
 *    [dx>=0] + 2[dy>=0] + 4[dz>=0], then the nearest others, truncated to
 *    m_max;
 *  - ghost mask: bit o ([sx>0] + 2[sy>0] + 4[sz>0]) set when no candidate
 *    lies beyond ghost_margin*h on every axis in octant s; each set bit
 *    adds a ghost row at offset h*s.
 * Stores them in the context for the fits.  Optional exports (null to
 * skip): cand_off (int64[n+1]) and cand_idx (int32[cap]) = candidate CSR
 * with ascending ids; needed (host) = total candidates (if cap is too
 * small nothing is written to cand_idx and LP_E_CAPACITY is returned);
 * sten_cnt (int32[n]) and sten_idx (int32[n*m_max], row-major, ascending
 * ids, padded with -1); ghost_mask (uint8[n]); n_mirror (host).  Exports
 * of cand_off/needed synchronise the stream. */
lp_status lp_neighbors(lp_ctx* ctx, const lp_state* s, int64_t* cand_off,
                       int32_t* cand_idx, int64_t cap, int64_t* needed,
                       int32_t* sten_cnt, int32_t* sten_idx,
                       uint8_t* ghost_mask, int64_t* n_mirror);

/* Second-order least-squares derivatives (Sec. 3.1 step 7, 3D): for each
 * real i and field q, minimises sum_rows w (a_r . c - (f_r - f_i))^2 with
 * Taylor rows a = (xi_x, xi_y, xi_z, xi_x^2/2, xi_y^2/2, xi_z^2/2,
 * xi_x xi_y, xi_x xi_z, xi_y xi_z), xi = (x_r - x_i)/h, over the stencil
 * and ghost rows (xi = s).  f: k x n (row-major, reals).  Mirror value =
 * mirror_sign[q] (host int32[k]) times the value at its source; ghost value
 * = f_i, or 0 when ghost_zero[q] (host int32[k]) is non-zero.  coef:
 * k x 9 x n (row-major): d/dx, d/dy, d/dz, d2/dx2, d2/dy2, d2/dz2,
 * d2/dxdy, d2/dxdz, d2/dydz.  flags (uint8[n], optional): bit0 linear
 * fallback (fewer than 9 rows or min|r_jj|/max|r_jj| < fallback_tol),
 * bit3 the stencil was refitted by Householder QR.  1 <= k <= 8. */
lp_status lp_fit_derivs(lp_ctx* ctx, const lp_state* s, const double* f,
                        int32_t k, const int32_t* mirror_sign,
                        const int32_t* ghost_zero, double* coef,
                        uint8_t* flags);

/* mu(I) closure and right-hand side from given velocity derivatives
 * coef_u (3 x 9 x n, layout of lp_fit_derivs for u, v, w):
 *   G_ab = d u_a/d x_b, D = (G + G^T)/2, gd = D - div/3 I,
 *   |gd| = sqrt(gd:gd/2), phi = 1/V; P and eta from eq. EOS2 with
 *   eta = mu(I) P/|gd| in the inertial branch (I = (phi_c - phi)/a), 0
 *   otherwise; mirrors carry P(phi_src, |gd| = 0) and eta = 0, ghosts 0;
 *   grad P and grad eta by the same fit (first derivatives);
 *   acc_a = V (-d_a P + gd_ab d_b eta + eta (Lap u_a/2 + d_a div u/6))
 *           / rho_s + g_a,   dVdt = V div u.
 * Outputs (device, any may be null except acc and dVdt): dVdt (n),
 * acc (3 x n), diag (5 x n: P, eta, I, mu, |gd|; I = mu = 0 off the
 * inertial branch), grad (6 x n: grad P, grad eta), flags (n: bit0 linear
 * fallback, bits1-2 branch 0 gas / 1 inertial / 2 quasi-static, bit3 QR
 * refit). */
lp_status lp_rheology_rhs(lp_ctx* ctx, const lp_state* s,
                          const double* coef_u, double* dVdt, double* acc,
                          double* diag, double* grad, uint8_t* flags);

/* Record of one step (lp_step or lp_step2) for its adjoint: which
 * particle order and which neighbour list the step used, so that
 * lp_step_adjoint / lp_step2_adjoint can differentiate that same step
 * without re-sorting or rebuilding the list.  Host struct owned by the
 * caller; perm is a caller-owned device array.
 *   force_sort (in):  1 makes the step re-sort and rebuild the list first
 *                     whatever the skin allows (a trajectory starts each
 *                     checkpointed segment this way, so that recomputing
 *                     the segment from its checkpoint reproduces it);
 *   resorted (out):   1 if the step re-sorted the state first, else 0;
 *   list_gen (out):   generation of the neighbour list the step used
 *                     (every list build makes a new generation);
 *   perm (device int32[n], required): receives perm[new] = old of the
 *                     re-sort when resorted = 1 (unwritten otherwise). */
typedef struct {
    int32_t force_sort;
    int32_t resorted;
    int64_t list_gen;
    int32_t* perm;
} lp_step_record;

/* One explicit step (Sec. 3.1 steps 5-10): when the context has no
 * neighbour list yet, or some particle has moved skin R / 2 since it was
 * built (checked on the device; one synchronisation), the state is
 * re-sorted as in lp_build_cells and the list rebuilt (perm as there);
 * otherwise the order is kept (perm, if given, is the identity).  Then
 * mirrors, stencils, fit of u, v, w, closure, fit of P and eta,
 * right-hand side, and
 *   V' = V + dt dVdt,  u' = u + dt acc,  x' = x + dt (u + u')/2.
 * The state must keep the order of the previous lp_step between calls.
 * rec (optional, null to skip): filled as described at lp_step_record;
 * with rec->force_sort = 1 the step re-sorts first.
 * dt > 0.  A non-finite result latches LP_E_NUMERIC (lp_sync_status). */
lp_status lp_step(lp_ctx* ctx, lp_state* s, double dt, int32_t* perm,
                  lp_step_record* rec);

/* One second-order step (Heun's predictor-corrector; the higher-order time
 * integration the conclusions list as further work, built from two
 * evaluations of the right-hand side f of Sec. 2.1 / Sec. 3.1 step 7):
 *   s* = s + dt f(s)   (x* = x + dt u, u* = u + dt acc, V* = V + dt dVdt)
 *   x' = x + dt (u + u*)/2,  u' = u + dt (acc(s) + acc(s*))/2,
 *   V' = V + dt (dVdt(s) + dVdt(s*))/2.
 * Mirrors and stencils are re-selected at s*, from the neighbour list of s.
 * Re-sort and list rebuild as in lp_step, but already once some particle
 * has moved 0.4 skin R since the build, so that the predictor stays within
 * half the skin; if some particle of s* is not, the step latches an error
 * that lp_sync_status reports as LP_E_STATE (reduce dt or raise skin).
 * Needs skin > 0 (LP_E_ARG otherwise).  State order, perm, dt and
 * non-finite results as for lp_step; the two kinds of step may alternate
 * on one state.  rec (optional) as for lp_step. */
lp_status lp_step2(lp_ctx* ctx, lp_state* s, double dt, int32_t* perm,
                   lp_step_record* rec);

/* Chooses how many adjacent lanes of a wavefront share one particle in
 * each of the two least-squares fit kernels (1, 2 or 4: each lane takes
 * every 1st, 2nd or 4th stencil row and the Gram moments are summed across
 * the lanes), by timing every choice on the stencils of s (not modified),
 * and, for float64 quadratic fits, whether to run the fits by stencil size
 * class with each class's fastest lanes per particle (lp_fit_plan).
 * lp_step, lp_step2, lp_step_graph and lp_rheology_rhs use the choice
 * afterwards.  choice (host int32[2], optional) receives the lanes per
 * particle of the first (u, v, w) and second (P, eta) fit as one launch.
 * Synchronises; leaves the context without a neighbour list and drops a
 * captured graph.  Results differ between choices only by summation
 * order. */
lp_status lp_autotune(lp_ctx* ctx, const lp_state* s, int32_t* choice);

/* The fit plan in use (batching of uneven stencils).  plan (host
 * int32[12]): [0], [1] lanes per particle of the first (u, v, w) and
 * second (P, eta) fit when each runs as one launch; [2] 1 when the float64
 * quadratic fits run instead by stencil size class (rows, ghosts
 * included: at most 16, at most 32, more), one launch per class over its
 * particles; [3..5], [6..8] lanes per particle of each class in the first
 * and second fit (0 on the largest class: the one-lane kernel over whole
 * tiles of particles with their neighbours staged in LDS, skipping the
 * smaller classes); [9..11] particles per class at the last lp_autotune.
 * ms (host double[8], optional): the best times lp_autotune measured,
 * milliseconds: [0], [1] one launch of each fit, [2..4], [5..7] each
 * class of the first and second fit (0 for an empty class).  lp_autotune
 * sets the plan (size classes when their total is the faster);
 * LP_DEBUG_CLASSES starts a context with size classes (lanes as listed
 * with the debug flags). */
lp_status lp_fit_plan(lp_ctx* ctx, int32_t* plan, double* ms);

/* nsteps consecutive lp_step calls as one HIP graph, for callers that
 * replay fixed step sequences without host work between steps.  Every
 * step decides on the device whether to re-sort and rebuild its neighbour
 * list (same rule as lp_step) and synchronises nothing.  The sequence is
 * captured on the first call (on a stream the library creates) and
 * replayed on the context's stream by later calls with the same state
 * arrays, ids, dt and nsteps (any change recaptures; lp_reserve drops the
 * capture).  ids (device int32[n], optional) are permuted along with the
 * state at every re-sort, so they track particle identity.  If the
 * context has no neighbour list, the state (and ids) are first re-sorted
 * in place as by lp_build_cells.  Between re-sorts the grid keeps the bit
 * budget it had at capture plus one bit per axis; beyond that cells are
 * enlarged (same results, more candidates tested).  dt > 0,
 * 1 <= nsteps <= 4096.  Asynchronous; device errors latch as for lp_step
 * (lp_sync_status). */
lp_status lp_step_graph(lp_ctx* ctx, lp_state* s, int32_t* ids, double dt,
                        int32_t nsteps);

/* Adjoint (reverse-mode derivative) of one step, for gradients of a loss
 * through the method (Sec. 3.1 steps 5-10 with the closure of Sec. 2.2 and
 * 2.2.1 and the right-hand side of Sec. 2.1).
 * Without a record (rec null) the step differentiated is lp_build_cells
 * followed by lp_step on s: s is re-sorted by the context's cells
 * (perm[new] = old, written to perm if not null), then stepped; the list
 * is rebuilt for this call and the next lp_step rebuilds again.
 * With the record of an lp_step (rec filled by lp_step on the same state
 * s), the step differentiated is that lp_step: s is put into the order
 * the step used (rec->perm when rec->resorted, else kept; perm receives
 * that permutation or the identity) and the step's neighbour list is
 * reused, which must still be the context's current list
 * (rec->list_gen; LP_E_STATE otherwise, e.g. after a later re-sort or
 * another call that rebuilt the list); the list stays valid afterwards.
 * Either way its
 * stencils, ghost masks, linear-fallback choices and regime branches are
 * held fixed (they are piecewise constant in the state); the shear-rate
 * norm is given zero derivative where it is zero.
 *   s:          the state before the step (device, caller's order; read);
 *   adj_out:    dL/d(state after the step), in the step's output order;
 *   adj_in:     receives dL/d(s) in s's order (overwritten; must not
 *               alias adj_out or s);
 *   adj_params: device double[n_sys x 3], dL/d(mu_s, mu_2, I0) per system
 *               is ADDED to it.
 * Computes in float64 whatever the precision setting; requires unit
 * weights (LP_E_ARG otherwise).  Neighbour contributions are summed per
 * tile of the neighbour list and added with float64 atomics (the
 * summation order, and so the rounding, varies between runs).  A
 * degenerate Gram matrix latches LP_E_NUMERIC (lp_sync_status). */
lp_status lp_step_adjoint(lp_ctx* ctx, const lp_state* s, double dt,
                          const lp_state* adj_out, lp_state* adj_in,
                          double* adj_params, int32_t* perm,
                          const lp_step_record* rec);

/* Adjoint of one second-order step: lp_build_cells followed by lp_step2 on
 * s (rec null), or the lp_step2 that filled rec, reversed through both
 * stages of Heun's rule with the stencils of s and
 * of the predictor s* held fixed (as lp_step_adjoint holds those of its
 * step):  with f = (u, acc, dVdt) and lam' = dL/d(s'),
 *   lam* = dL/d(s*) = J_f(s*)^T (dt/2 lam'),
 *   dL/d(s) = lam' + lam* + J_f(s)^T (dt (lam'/2 + lam*)).
 * Arguments, orders, records, float64 arithmetic, unit weights, capacity
 * limit and the effect on the context as for lp_step_adjoint; needs
 * skin > 0, and the
 * predictor must stay within half the skin (else the error latches as in
 * lp_step2).  Recomputes the forward stages (pass 1 at s twice, once at
 * s*). */
lp_status lp_step2_adjoint(lp_ctx* ctx, const lp_state* s, double dt,
                           const lp_state* adj_out, lp_state* adj_in,
                           double* adj_params, int32_t* perm,
                           const lp_step_record* rec);

/* Allocation-free step, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): one lp_step on a fresh context with configuration
 * cfg (null: defaults) and the given systems (n_sys, host offsets and
 * params as for lp_set_systems) on `stream`, i.e. re-sort and list build
 * (perm[new] = old, optional), stencils, fits, closure, right-hand side
 * and update of s in place, then lp_sync_status.  No context is created
 * and nothing is allocated: the workspace is a static device array of
 * about 46 MB (44 MiB) that each device the library runs on holds until the
 * process ends, set up on a device's first call.  Limits: at most 16384
 * particles, 64 systems and 65536 cells; beyond them LP_E_CAPACITY (the
 * particle and system counts are checked before any work is enqueued).
 * Returns LP_E_ARG for invalid arguments or configuration, and the status
 * lp_sync_status would give for device-side errors (no text: there is no
 * context to hold it).  Every call on a device shares that device's
 * array, so calls that overlap on one device race (the library serialises
 * host threads, not streams); each call clears what it needs and keeps
 * nothing from the previous call.  Synchronises `stream`. */
lp_status lp_step_noalloc(void* stream, const lp_config* cfg, int32_t n_sys,
                          const int64_t* offsets, const lp_params* params,
                          lp_state* s, double dt, int32_t* perm);

/* Synchronises the context's stream and returns the first latched device
 * error (LP_OK if none), then clears it.  *index (host, optional)
 * receives the first offending particle or -1. */
lp_status lp_sync_status(lp_ctx* ctx, int64_t* index);

/* Diagnostics accumulated since the last call (host int64[8]):
 * particles, mirrors (last stencil build), QR refits, sorted-path stencils,
 * particles below the wall after updates, neighbour-list rebuilds by
 * lp_step; then resets them.  Entries 6 and 7 describe the current
 * neighbour list (0 when there is none): tiles of BLOCK = 256 consecutive
 * particles whose neighbours the fits cannot stage in LDS (more than 1664
 * distinct list sources, LP_DEBUG_GLOBAL_GATHER, or every tile while the
 * list has no tile map: the map is built by lp_step, lp_step2 and
 * lp_step_graph, not by lp_build_cells or the adjoint entry points), and
 * all tiles.
 * Synchronises. */
lp_status lp_stats(lp_ctx* ctx, int64_t* out8);

/* Phase timing (instrumentation).  lp_profile(ctx, 1) makes lp_step
 * record HIP events on the context's stream around its kernel groups:
 * 0 displacement check and re-sort + list rebuild (with its tile map) or
 * state copy, 1 stencil selection (k_select alone; the mirror kernels
 * before it are in no phase), 2 exact sorted-stencil path, 3 pass-1 fit +
 * closure (k_pass1_st), 4 pass-1 QR refits, 5 pass-2 fit + RHS + update
 * (k_pass2_st), 6 pass-2 QR refits; each lp_step then
 * waits for its last event.  lp_profile_read (host double[8], int64 steps)
 * returns the summed milliseconds per phase and the number of profiled
 * steps, then resets them.  lp_profile(ctx, 0) stops recording. */
lp_status lp_profile(lp_ctx* ctx, int32_t enable);
lp_status lp_profile_read(lp_ctx* ctx, double* ms8, int64_t* steps);

#ifdef __cplusplus
}
#endif

#endif /* LP_H */
