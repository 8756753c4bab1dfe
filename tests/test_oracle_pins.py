"""Pins of the FP64 CPU oracle against facts fixed by the paper, by
mathematics or by independent library routines (no GPU needed).

Each test states what it pins.  A plausible mistake in the oracle (a
dropped term, a wrong sign or index, a transposed operand, a wrong
stencil rule) fails at least one of them.
"""
import math

import numpy as np
import pytest

import lpgen
import oracle
from lpgen import Params, State

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _state_from_points(pts, u=None, V=None):
    n = pts.shape[0]
    z = np.zeros(n)
    u = np.zeros((n, 3)) if u is None else u
    V = np.full(n, 1.0 / 0.45) if V is None else V
    return State(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(),
                 u[:, 0].copy(), u[:, 1].copy(), u[:, 2].copy(), V.copy())


def _one(state, p, **kw):
    return oracle.Oracle(state, np.array([0, state.n]), [p], **kw)


# ----------------------------------------------------------------------
# Morton order
# ----------------------------------------------------------------------

def _interleave_by_strings(cx, cy, cz, bits=21):
    """Morton code built from binary strings: the k-th bit triple (from the
    least significant end) is (z_k y_k x_k)."""
    bx, by, bz = (format(v, "0%db" % bits) for v in (cx, cy, cz))
    s = "".join(bz[i] + by[i] + bx[i] for i in range(bits))
    return int(s, 2)


def test_morton_keys_are_bit_interleaves():
    """Cell keys are the x/y/z bit interleave of the cell coordinates."""
    h = 0.1
    p = lpgen.default_params(h)
    c = (p.R * (1.0 + oracle.SKIN_DEFAULT)) * (1.0 + 2.0 ** -20)
    p.wall_z = 0.0 + p.R          # wall - R = 0 = lowest particle cell edge
    cells = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (3, 0, 0),
             (1, 1, 1), (5, 2, 7), (12, 9, 3), (2, 6, 1)]
    pts = np.array([[(cx + 0.5) * c, (cy + 0.5) * c, (cz + 0.5) * c]
                    for cx, cy, cz in cells])
    pts[0] = [0.0, 0.0, 0.0]       # defines the origin
    st = _state_from_points(pts)
    perm, keys = oracle.sort_perm(st, np.array([0, st.n]), [p])
    want = {}
    for k, (cx, cy, cz) in enumerate(cells):
        want[k] = _interleave_by_strings(cx, cy, cz)
    got = {int(perm[i]): int(keys[i]) for i in range(st.n)}
    assert got == want
    assert [_interleave_by_strings(*c_) for c_ in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]] == [1, 2, 4]


def test_sort_is_stable_permutation():
    """perm is a permutation; keys are non-decreasing and equal keys keep
    the old index order (stable)."""
    rng = np.random.default_rng(7)
    pts = rng.uniform(0, 0.6, size=(3000, 3))
    pts[:500] = pts[:1][0] + rng.uniform(0, 1e-3, size=(500, 3))  # many ties
    st = _state_from_points(pts)
    p = lpgen.default_params(0.05)
    perm, keys = oracle.sort_perm(st, np.array([0, st.n]), [p])
    assert np.array_equal(np.sort(perm), np.arange(st.n))
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    same = keys[1:] == keys[:-1]
    assert np.all(perm[1:][same] > perm[:-1][same])


# ----------------------------------------------------------------------
# Mirrors, neighbours, stencils, ghosts
# ----------------------------------------------------------------------

def test_mirrors_reflect_across_wall():
    """Sec. 3.1 step 9: one mirror per particle closer than R to the wall,
    at (x, y, 2 z_w - z), velocity (u, v, -w), same V, ascending source."""
    wl = lpgen.column_small()
    st = wl.state
    rng = np.random.default_rng(3)
    st.u = rng.normal(size=st.n)
    st.v = rng.normal(size=st.n)
    st.w = rng.normal(size=st.n)
    p = wl.params[0]
    o = _one(st, p)
    nb = o.neighbours()
    src = np.nonzero(st.z - p.wall_z < p.R)[0]
    assert nb.n_mirror == src.size
    assert np.array_equal(nb.mirror_src, src)
    m = nb.mirror_state
    assert np.array_equal(m[0], st.x[src]) and np.array_equal(m[1], st.y[src])
    assert np.array_equal(m[2], 2.0 * p.wall_z - st.z[src])
    assert np.array_equal(m[3], st.u[src]) and np.array_equal(m[4], st.v[src])
    assert np.array_equal(m[5], -st.w[src]) and np.array_equal(m[6], st.V[src])


def _all_points(st, nb):
    m = nb.mirror_state
    return np.concatenate([np.stack([st.x, st.y, st.z], 1), m[:3].T], axis=0)


def test_neighbours_match_kdtree():
    """Candidate sets equal an independent KD-tree ball query (scipy),
    except pairs within 1e-9 R of the cut radius, where the two distance
    formulas may round differently."""
    from scipy.spatial import cKDTree
    wl = lpgen.column_small()
    st, p = wl.state, wl.params[0]
    o = _one(st, p)
    nb = o.neighbours()
    pts = _all_points(st, nb)
    tree = cKDTree(pts)
    lists = tree.query_ball_point(pts[:st.n], p.R)
    for i in range(0, st.n, 7):
        mine = set(nb.cand_idx[nb.cand_off[i]:nb.cand_off[i + 1]].tolist())
        ref = set(lists[i]) - {i}
        diff = mine ^ ref
        for j in diff:
            r = np.linalg.norm(pts[j] - pts[i])
            assert abs(r - p.R) < 1e-9 * p.R, (i, j, r)
        assert list(nb.cand_idx[nb.cand_off[i]:nb.cand_off[i + 1]]) == sorted(mine)


@pytest.mark.parametrize("kind", ["lattice", "sheared"])
def test_cell_list_equals_brute_force(kind):
    """The oracle's bucket-grid search returns exactly the O(N^2) sets."""
    if kind == "lattice":
        st = lpgen.column_small().state
        p = lpgen.column_small().params[0]
    else:
        wl = lpgen.column_sheared(nx=14, ny=14, nz=10)
        st, p = wl.state, wl.params[0]
    a = _one(st, p, brute=True).neighbours()
    b = _one(st, p, brute=False).neighbours()
    assert np.array_equal(a.cand_off, b.cand_off)
    assert np.array_equal(a.cand_idx, b.cand_idx)
    assert np.array_equal(a.sten_idx, b.sten_idx)
    assert np.array_equal(a.ghost_mask, b.ghost_mask)


def test_candidate_test_rounds_like_the_plain_definition():
    """Pairs on the cut radius to the last bit: the oracle's candidate test
    follows r2 = (dx*dx + dy*dy) + dz*dz with every operation rounded (no
    fused multiply-add), checked against numpy float64 arithmetic."""
    from rounding_cases import straddle_workload, unfused_r2
    wl, want = straddle_workload()
    o = oracle.Oracle(wl.state, wl.offsets, wl.params, brute=True)
    nb = o.neighbours()
    for s, inside in enumerate(want):
        i = 2 * s
        cand = nb.cand_idx[nb.cand_off[i]:nb.cand_off[i + 1]]
        assert (i + 1 in cand) == inside
        d = np.array([wl.state.x[i + 1] - wl.state.x[i], wl.state.y[i + 1] - wl.state.y[i],
                      wl.state.z[i + 1] - wl.state.z[i]])
        assert (unfused_r2(*d) < wl.params[s].R * wl.params[s].R) == inside


def _keys(st, nb, i, ids):
    pts = _all_points(st, nb)
    d = pts[ids] - pts[i]
    r2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    octs = (d[:, 0] >= 0).astype(int) + 2 * (d[:, 1] >= 0) + 4 * (d[:, 2] >= 0)
    return r2, octs


@pytest.mark.parametrize("kind", ["lattice", "sheared"])
def test_stencil_invariants(kind):
    """Sec. 3.1 step 6: the stencil holds the nearest candidate of every
    occupied octant, then the nearest others, min(count, m_max) in all;
    every dropped candidate is farther (key (r2, id)) than every kept
    non-octant-first candidate."""
    if kind == "lattice":
        wl = lpgen.column_small()
    else:
        wl = lpgen.column_sheared(nx=14, ny=14, nz=10)
    st, p = wl.state, wl.params[0]
    o = _one(st, p)
    nb = o.neighbours()
    mm = o.m_max
    for i in range(0, st.n, 3):
        cand = nb.cand_idx[nb.cand_off[i]:nb.cand_off[i + 1]]
        k = nb.sten_cnt[i]
        sten = nb.sten_idx[i, :k]
        assert k == min(cand.size, mm)
        assert set(sten.tolist()) <= set(cand.tolist())
        assert len(set(sten.tolist())) == k
        r2, octs = _keys(st, nb, i, cand)
        order = sorted(range(cand.size), key=lambda t: (r2[t], cand[t]))
        firsts = {}
        for t in order:
            firsts.setdefault(octs[t], cand[t])
        assert set(firsts.values()) <= set(sten.tolist())
        # canonical order: octant-firsts in octant order first
        fo = [firsts[q] for q in sorted(firsts)]
        assert list(sten[:len(fo)]) == fo
        kept = set(sten.tolist()) - set(firsts.values())
        dropped = set(cand.tolist()) - set(sten.tolist())
        if kept and dropped:
            kk = max((r2[list(cand).index(j)], j) for j in kept)
            dd = min((r2[list(cand).index(j)], j) for j in dropped)
            assert kk < dd


def test_octant_first_survives_truncation():
    """A lone neighbour in an otherwise empty octant stays in the stencil
    even when 70 nearer neighbours crowd another octant (the paper's rule
    that the top entries cover all directions)."""
    h = 0.1
    p = lpgen.default_params(h)
    p.wall_z = -100.0
    rng = np.random.default_rng(11)
    crowd = rng.uniform(0.05, 0.55, size=(70, 3)) * p.R / math.sqrt(3) * 1.5
    crowd = np.abs(crowd)
    lone = np.array([[-0.5, -0.5, -0.55]]) * p.R
    pts = np.concatenate([np.zeros((1, 3)), crowd, lone]) + 5.0
    st = _state_from_points(pts)
    o = _one(st, p)
    nb = o.neighbours()
    lone_id = pts.shape[0] - 1
    cand = nb.cand_idx[nb.cand_off[0]:nb.cand_off[1]]
    assert lone_id in cand and cand.size == 71
    assert nb.sten_cnt[0] == 60
    assert lone_id in nb.sten_idx[0, :60]
    assert nb.sten_idx[0, 0] == lone_id     # octant 0 comes first


def test_ghost_masks_on_column_faces():
    """Sec. 3.1 steps 5/9: interior particles and particles on the wall
    (mirrors complete them) get no ghost; the top face gets the four
    upper octants; the top corner at max x, max y gets all but (-,-,-);
    an isolated particle gets all eight."""
    wl = lpgen.column_small()
    st, p = wl.state, wl.params[0]
    o = _one(st, p)
    nb = o.neighbours()
    h = p.h
    ids = np.arange(st.n)
    i = ids % 16
    j = (ids // 16) % 16
    k = ids // 256
    interior = (i >= 3) & (i <= 12) & (j >= 3) & (j <= 12) & (k <= 12)
    assert np.all(nb.ghost_mask[interior] == 0)
    top = (i >= 3) & (i <= 12) & (j >= 3) & (j <= 12) & (k == 15)
    assert np.all(nb.ghost_mask[top] == 0xF0)
    corner = (i == 15) & (j == 15) & (k == 15)
    assert np.all(nb.ghost_mask[corner] == 0xFE)
    # isolated particle, far from the wall
    p2 = lpgen.default_params(h)
    st2 = _state_from_points(np.array([[0.0, 0.0, 3.0]]), V=np.array([1 / 0.3]))
    nb2 = _one(st2, p2).neighbours()
    assert nb2.ghost_mask[0] == 0xFF and nb2.sten_cnt[0] == 0


# ----------------------------------------------------------------------
# Least squares
# ----------------------------------------------------------------------

def test_lsq_matches_lapack_svd_solver():
    """Householder QR least squares equals numpy.linalg.lstsq (LAPACK
    gelsd, an SVD method) on random tall systems."""
    rng = np.random.default_rng(5)
    for m in (9, 10, 17, 40, 68):
        A = rng.normal(size=(m, 9))
        B = rng.normal(size=(m, 4))
        Cq, ratio = oracle.lsq(A, B)
        Cs = np.linalg.lstsq(A, B, rcond=None)[0]
        assert np.max(np.abs(Cq - Cs)) <= 1e-12 * np.max(np.abs(Cs))
        assert ratio > 1e-3


def test_lsq_detects_rank_deficiency():
    """A repeated column drives min|r_jj|/max|r_jj| to rounding level."""
    rng = np.random.default_rng(6)
    A = rng.normal(size=(20, 9))
    A[:, 5] = A[:, 4]
    _, ratio = oracle.lsq(A, rng.normal(size=(20, 1)))
    assert ratio < 1e-12


def _quad_fields(rng, pts, nf=4):
    """Random quadratics f = c0 + g.x + x^T H x / 2 with exact derivatives."""
    F, D = [], []
    for _ in range(nf):
        c0 = rng.normal()
        g = rng.normal(size=3)
        Hs = rng.normal(size=(3, 3))
        Hs = Hs + Hs.T
        f = c0 + pts @ g + 0.5 * np.einsum("ni,ij,nj->n", pts, Hs, pts)
        grad = g[None, :] + pts @ Hs
        F.append(f)
        D.append((grad, Hs))
    return np.array(F), D


@pytest.mark.parametrize("layout", ["lattice", "random", "sheared"])
def test_fit_reproduces_quadratics(layout):
    """Sec. 3.1 step 7: the 2nd-order fit is exact for polynomials of
    degree <= 2 (stencils without ghost rows)."""
    rng = np.random.default_rng({"lattice": 1, "random": 2, "sheared": 3}[layout])
    h = 0.05
    p = lpgen.default_params(h)
    p.wall_z = -100.0
    if layout == "random":
        pts = rng.uniform(0, 12 * h, size=(1728, 3))
    else:
        st0 = lpgen.lattice_column(12, 12, 12, h, seed=99, params=p)
        pts = np.stack([st0.x, st0.y, st0.z], 1)
        if layout == "sheared":
            pts = pts @ np.array([[1.0, 0.0, 0.0], [0.3, 1.0, 0.0], [0.2, -0.25, 1.0]])
    pts = pts + np.array([0.3, -0.2, 0.1])
    st = _state_from_points(pts)
    o = _one(st, p)
    nb = o.neighbours()
    F, D = _quad_fields(rng, pts)
    coef, flags = o.fit(F, [1] * 4, [0] * 4)
    ok = (nb.ghost_mask == 0) & (flags == 0)
    assert ok.sum() > 50
    for f, (grad, Hs) in enumerate(D):
        scale = np.max(np.abs(grad)) + np.max(np.abs(Hs))
        for a in range(3):
            err = np.abs(coef[f, a, ok] - grad[ok, a])
            assert err.max() <= 1e-12 * scale
        for c, (a, b) in enumerate([(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]):
            err = np.abs(coef[f, 3 + c, ok] - Hs[a, b])
            assert err.max() <= 1e-11 * scale


def test_fit_matches_lapack_on_stencil_rows():
    """The per-particle fit equals a LAPACK least-squares solve of the
    exported stencil's Taylor rows (arbitrary, non-polynomial data)."""
    wl = lpgen.column_small()
    st, p = wl.state, wl.params[0]
    rng = np.random.default_rng(8)
    f = rng.normal(size=st.n)
    o = _one(st, p)
    nb = o.neighbours()
    coef, flags = o.fit(f[None, :], [1], [0])
    pts = _all_points(st, nb)
    fa = np.concatenate([f, f[nb.mirror_src]])
    for i in range(0, st.n, 97):
        ids = nb.sten_idx[i, :nb.sten_cnt[i]]
        d = (pts[ids] - pts[i]) / p.h
        rows = [np.array([e[0], e[1], e[2], e[0] ** 2 / 2, e[1] ** 2 / 2,
                          e[2] ** 2 / 2, e[0] * e[1], e[0] * e[2], e[1] * e[2]])
                for e in d]
        b = list(fa[ids] - f[i])
        for q in range(8):
            if nb.ghost_mask[i] >> q & 1:
                s = [1.0 if q & 1 else -1.0, 1.0 if q & 2 else -1.0,
                     1.0 if q & 4 else -1.0]
                rows.append(np.array([s[0], s[1], s[2], .5, .5, .5, s[0] * s[1],
                                      s[0] * s[2], s[1] * s[2]]))
                b.append(0.0)
        A = np.array(rows)
        c = np.linalg.lstsq(A, np.array(b), rcond=None)[0]
        c[:3] /= p.h
        c[3:] /= p.h ** 2
        assert flags[i] == 0
        assert np.max(np.abs(coef[0, :, i] - c)) <= 1e-10 * np.max(np.abs(c))


def test_fit_convergence_order():
    """Observed order on a smooth field with fixed relative jitter, over
    three refinements: gradient >= 1.8, second derivatives >= 0.9 (a
    second-order fit; with jittered points the second derivatives are
    first-order accurate)."""
    errs1, errs2, hs = [], [], []
    L = 0.6
    for nl in (12, 24, 48):
        h = L / nl
        p = lpgen.default_params(h)
        p.wall_z = -100.0
        st0 = lpgen.lattice_column(nl, nl, nl, h, seed=5, params=p)
        pts = np.stack([st0.x, st0.y, st0.z], 1)
        k = np.array([3.0, 2.0, 2.5])
        f = np.sin(pts @ k) + np.cos(2.0 * pts[:, 0] - pts[:, 2])
        gx = np.cos(pts @ k)[:, None] * k[None, :]
        gx[:, 0] += -2.0 * np.sin(2.0 * pts[:, 0] - pts[:, 2])
        gx[:, 2] += np.sin(2.0 * pts[:, 0] - pts[:, 2])
        hxx = -np.sin(pts @ k) * k[0] ** 2 - 4.0 * np.cos(2.0 * pts[:, 0] - pts[:, 2])
        st = _state_from_points(pts)
        o = _one(st, p)
        coef, flags = o.fit(f[None, :], [1], [0])
        c = np.array([L / 2] * 3)
        inner = np.all(np.abs(pts - c) < 0.15, axis=1)
        assert np.all(o.neighbours().ghost_mask[inner] == 0)
        errs1.append(np.max(np.abs(coef[0][:3][:, inner].T - gx[inner])))
        errs2.append(np.max(np.abs(coef[0, 3, inner] - hxx[inner])))
        hs.append(h)
    # observed order = least-squares slope of log(err) against log(h)
    o1 = np.polyfit(np.log(hs), np.log(errs1), 1)[0]
    o2 = np.polyfit(np.log(hs), np.log(errs2), 1)[0]
    assert o1 >= 1.8, (errs1, o1)
    assert o2 >= 0.9, (errs2, o2)


# ----------------------------------------------------------------------
# Closure
# ----------------------------------------------------------------------

def _inertial_phi(p, I):
    return p.phi_c - (p.phi_c - p.phi_min) * I


def test_simple_shear_gives_textbook_inertial_number():
    """For simple shear u = (s y, 0, 0) the shear-rate norm is s/2, so the
    paper's I = 2|gd| d / sqrt(P/rho_s) is the usual s d / sqrt(P/rho_s);
    and that I equals (phi_c - phi)/a (eqs. inertial, inertialdensity)."""
    p = Params()
    s = 7.5
    G = np.array([[0.0, s, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    for phi in (0.36, 0.45, 0.53025, 0.589):
        br, P, eta, I, mu, gn, gd = oracle.closure_point(p, 1.0 / phi, G)
        assert br == oracle.BR_INERTIAL
        assert abs(gn - s / 2) <= 1e-15 * s
        I_text = s * p.d / math.sqrt(P / p.rho_s)
        assert abs(I_text - I) <= 1e-12 * I
        assert abs(I - (p.phi_c - phi) / (p.phi_c - p.phi_min)) <= 1e-12 * I


def test_mu_of_I_closed_forms():
    """mu(I0) is the midpoint of mu_s and mu_2; |tau| = eta |gd| = mu P
    (eqs. friction, align, CST1); with the paper's own constants too."""
    for p in (Params(), Params(mu_s=math.tan(math.radians(30)),
                               mu_2=math.tan(math.radians(50)), I0=2.65,
                               d=0.32e-3, rho_s=2600.0)):
        phi = _inertial_phi(p, p.I0) if p.I0 < 0.9 else 0.45
        rng = np.random.default_rng(1)
        G = rng.normal(size=(3, 3))
        br, P, eta, I, mu, gn, gd = oracle.closure_point(p, 1.0 / phi, G)
        assert br == oracle.BR_INERTIAL
        if p.I0 < 0.9:
            assert abs(mu - 0.5 * (p.mu_s + p.mu_2)) <= 1e-14
        want = p.mu_s + (p.mu_2 - p.mu_s) * I / (p.I0 + I)
        assert abs(mu - want) <= 1e-14
        assert abs(eta * gn - mu * P) <= 1e-12 * mu * P
        assert p.mu_s < mu < p.mu_2


def test_closure_matches_M_N_forms():
    """Sec. 2.3: sigma/rho_s = M |gd|^2 delta + N |gd| gd with the printed
    M(phi) and N(phi), i.e. -P/rho_s = M |gd|^2 and eta/rho_s = N |gd|."""
    p = Params()
    a = p.phi_c - p.phi_min
    rng = np.random.default_rng(2)
    for phi in (0.37, 0.44, 0.5, 0.58):
        G = rng.normal(size=(3, 3))
        br, P, eta, I, mu, gn, gd = oracle.closure_point(p, 1.0 / phi, G)
        w = p.phi_c - phi
        M = -4 * a * a * p.d ** 2 / w ** 2
        N = 4 * a * a * p.d ** 2 / w ** 2 * (a * p.mu_s * p.I0 + p.mu_2 * w) / (a * p.I0 + w)
        assert abs(-P / p.rho_s - M * gn * gn) <= 1e-12 * abs(M) * gn * gn
        assert abs(eta / p.rho_s - N * gn) <= 1e-12 * N * gn


def test_shear_rate_tensor_properties():
    """gd is symmetric and trace free; |gd| is invariant under rotation of
    the velocity gradient (G -> Q G Q^T)."""
    p = Params()
    rng = np.random.default_rng(4)
    G = rng.normal(size=(3, 3))
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    _, _, _, _, _, gn, gd = oracle.closure_point(p, 1 / 0.45, G)
    _, _, _, _, _, gn2, _ = oracle.closure_point(p, 1 / 0.45, Q @ G @ Q.T)
    assert np.allclose(gd, gd.T, atol=1e-15) and abs(np.trace(gd)) < 1e-14
    assert abs(gn - gn2) <= 1e-13 * gn


def test_regime_branches_and_continuity():
    """EOS2: gas at phi <= phi_min (P = eta = 0), inertial on
    (phi_min, phi_max], quasi-static above with P = rho_s (alpha + beta
    phi); with alpha = -beta phi_max the pressure is continuous at phi_max
    for zero shear."""
    p = Params()
    G0 = np.zeros((3, 3))
    G = np.array([[0.0, 2.0, 0.0], [0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    assert oracle.closure_point(p, 1.0 / p.phi_min, G)[0] == oracle.BR_GAS
    assert oracle.closure_point(p, 1.0 / 0.2, G)[1:3] == (0.0, 0.0)
    assert oracle.closure_point(p, 1.0 / 0.35000001, G)[0] == oracle.BR_INERTIAL
    assert oracle.closure_point(p, 1.0 / p.phi_max, G)[0] == oracle.BR_INERTIAL
    br, P, eta, *_ = oracle.closure_point(p, 1.0 / 0.595, G)
    assert br == oracle.BR_QUASI and eta == 0.0
    assert abs(P - p.rho_s * p.beta * (0.595 - p.phi_max)) <= 1e-9 * P
    br, P, *_ = oracle.closure_point(p, 1.0 / (p.phi_max + 1e-12), G0)
    assert br == oracle.BR_QUASI and abs(P) < 1e-5
    assert oracle.closure_point(p, 1.0 / p.phi_max, G0)[1] == 0.0


# ----------------------------------------------------------------------
# Right-hand side and update
# ----------------------------------------------------------------------

def test_isolated_gas_particle_falls_freely():
    """A particle with no neighbours in the gas regime feels only gravity:
    a = g exactly, dV/dt = 0; the fit falls back to linear (8 ghost rows)."""
    p = lpgen.default_params(0.05)
    st = _state_from_points(np.array([[0.1, 0.2, 4.0]]), u=np.array([[1.0, -2.0, 0.5]]),
                            V=np.array([1.0 / 0.3]))
    r = _one(st, p).evaluate()
    assert np.array_equal(r["acc"][:, 0], np.array(p.g))
    assert r["dVdt"][0] == 0.0
    assert r["flags"][0] & oracle.FLAG_LINEAR


def test_update_by_hand():
    """Sec. 3.1 steps 8 and 10 for one free-falling particle, computed by
    hand: V' = V, u' = u + dt g, x' = x + dt (u + u')/2 (gravity on all
    three axes so that every component is exercised)."""
    p = lpgen.default_params(0.05, g=(1.5, -2.0, -9.81))
    x0 = np.array([0.1, 0.2, 4.0])
    u0 = np.array([1.0, -2.0, 0.5])
    st = _state_from_points(x0[None, :], u=u0[None, :], V=np.array([1.0 / 0.3]))
    dt = 1e-3
    new, perm, r = oracle.step(st, np.array([0, 1]), [p], dt)
    u1 = u0 + dt * np.array(p.g)
    x1 = x0 + dt * (0.5 * (u0 + u1))
    assert np.array_equal(np.array([new.u[0], new.v[0], new.w[0]]), u1)
    assert np.array_equal(np.array([new.x[0], new.y[0], new.z[0]]), x1)
    assert new.V[0] == 1.0 / 0.3


def test_uniform_slab_on_wall_feels_only_gravity():
    """A quasi-static slab of uniform density resting on the wall: mirrors
    carry the source's pressure (Sec. 3.1 step 9), so P is uniform across
    the wall and every particle more than R below the free top surface and
    away from the sides has a = g (to rounding)."""
    wl = lpgen.column_small()
    st, p = wl.state, wl.params[0]
    st.V[:] = 1.0 / 0.595
    r = _one(st, p).evaluate()
    H = 16 * p.h
    ok = ((st.x > p.R) & (st.x < 1.0 - p.R) & (st.y > p.R) & (st.y < 1.0 - p.R)
          & (st.z < H - p.R))
    near_wall = ok & (st.z < p.R)
    assert near_wall.sum() > 100
    P = p.rho_s * p.beta * (0.595 - p.phi_max)
    assert np.max(np.abs(r["acc"][:, ok] - np.array(p.g)[:, None])) <= 1e-10 * P


def test_hydrostatic_column_interior_at_rest():
    """The hydrostatic quasi-static column (phi = phi_max exp(g (H-z)/beta))
    is an equilibrium: interior particles (more than R from every free
    surface and from the wall) have |a| <= 1e-5 m/s^2."""
    wl = lpgen.column_small()
    st, p = wl.state, wl.params[0]
    r = _one(st, p).evaluate()
    H = 16 * p.h
    far = ((st.x > p.R) & (st.x < 1.0 - p.R) & (st.y > p.R) & (st.y < 1.0 - p.R)
           & (st.z > p.R) & (st.z < H - p.R))
    assert far.sum() > 500
    assert np.all((r["flags"][far] >> 1) == oracle.BR_QUASI)
    assert np.max(np.abs(r["acc"][:, far])) <= 1e-5


def _lattice_with_flow():
    """Jittered 16^3 lattice column with a smooth velocity field and a
    density field that visits the gas, inertial and quasi-static branches."""
    wl = lpgen.column_small()
    st, p = wl.state, wl.params[0]
    st.u = 0.3 * np.sin(3.1 * st.y + 1.0) * np.cos(2.0 * st.z)
    st.v = 0.2 * np.cos(2.3 * st.x) * np.sin(1.7 * st.z + 0.4)
    st.w = 0.25 * np.sin(2.9 * st.x + 1.1 * st.y)
    st.V = 1.0 / (0.47 + 0.15 * np.sin(4.0 * st.z + 2.0 * st.y))
    return st, p


def test_x_reflection_symmetry():
    """Reflecting the input x -> W - x (with u -> -u) reflects the RHS:
    a_x changes sign, a_y, a_z and dV/dt do not."""
    st, p = _lattice_with_flow()
    r1 = _one(st, p).evaluate()
    br = r1["flags"] >> 1
    assert set(np.unique(br).tolist()) == {0, 1, 2}
    W = 0.37
    st2 = State(W - st.x, st.y.copy(), st.z.copy(), -st.u, st.v.copy(),
                st.w.copy(), st.V.copy())
    r2 = _one(st2, p).evaluate()
    sc = np.max(np.abs(r1["acc"] - np.array(p.g)[:, None]))
    assert np.max(np.abs(r1["acc"][0] + r2["acc"][0])) <= 1e-10 * sc
    assert np.max(np.abs(r1["acc"][1:] - r2["acc"][1:])) <= 1e-10 * sc
    assert np.max(np.abs(r1["dVdt"] - r2["dVdt"])) <= 1e-10 * np.max(np.abs(r1["dVdt"]))


def test_galilean_invariance():
    """Adding a uniform horizontal velocity (U, W, 0) to every particle
    (mirrors included) leaves the RHS unchanged."""
    st, p = _lattice_with_flow()
    r1 = _one(st, p).evaluate()
    st2 = st.copy()
    st2.u = st2.u + 0.7
    st2.v = st2.v - 1.3
    r2 = _one(st2, p).evaluate()
    sc = np.max(np.abs(r1["acc"] - np.array(p.g)[:, None]))
    assert np.max(np.abs(r1["acc"] - r2["acc"])) <= 1e-9 * sc


def _manufactured(pts, p, kind="general"):
    """Analytic RHS of a smooth inertial-only field, by float64 autodiff of
    the continuum equations (no least squares involved).

    ``general``: every term of the momentum equation is active.
    ``viscous``: uniform density, a base shear u = s y plus a compressive
    x-wave A sin(kx) whose strain is orthogonal to the base shear, so grad P
    and grad eta are second order in A and the stress divergence is
    dominated by eta (Lap u / 2 + grad div u / 6)."""
    import torch
    X = torch.tensor(pts, dtype=torch.float64, requires_grad=True)
    s, A, k = 10.0, 0.1, 2 * math.pi / 0.5
    if kind == "viscous":
        A = 0.8

    def vel(X):
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        if kind == "viscous":
            zero = torch.zeros_like(x)
            return torch.stack([s * y + A * torch.sin(k * x), zero, zero], 1)
        return torch.stack([s * y + A * torch.sin(k * x) * torch.cos(k * z),
                            A * torch.cos(k * y) * torch.sin(k * x),
                            A * torch.sin(k * z) * torch.cos(k * y)], 1)

    def phi_of(X):
        x, y, z = X[:, 0], X[:, 1], X[:, 2]
        if kind == "viscous":
            return 0.47 + 0.0 * x
        return 0.47 + 0.05 * torch.sin(k * x + 0.3) * torch.cos(k * y) + 0.02 * torch.cos(k * z)

    U = vel(X)
    G = torch.stack([torch.autograd.grad(U[:, a].sum(), X, create_graph=True)[0]
                     for a in range(3)], 1)          # G[n, a, b] = d u_a / d x_b
    div = G[:, 0, 0] + G[:, 1, 1] + G[:, 2, 2]
    D = 0.5 * (G + G.transpose(1, 2))
    gd = D - div[:, None, None] / 3 * torch.eye(3, dtype=torch.float64)[None]
    gn = torch.sqrt(0.5 * (gd * gd).sum((1, 2)))
    phi = phi_of(X)
    a = p.phi_c - p.phi_min
    w = p.phi_c - phi
    P = p.rho_s * (2 * a * p.d * gn / w) ** 2
    I = w / a
    mu = p.mu_s + (p.mu_2 - p.mu_s) / (p.I0 / I + 1)
    eta = mu * P / gn
    sig = -P[:, None, None] * torch.eye(3, dtype=torch.float64)[None] + eta[:, None, None] * gd
    divs = torch.zeros(pts.shape[0], 3, dtype=torch.float64)
    for i in range(3):
        for j in range(3):
            g = torch.autograd.grad(sig[:, i, j].sum(), X, retain_graph=True)[0]
            divs[:, i] = divs[:, i] + g[:, j]
    acc = divs / (p.rho_s * phi[:, None]) + torch.tensor(p.g, dtype=torch.float64)[None]
    dVdt = div / phi
    return (U.detach().numpy(), (1.0 / phi).detach().numpy(),
            acc.detach().numpy(), dVdt.detach().numpy())


@pytest.mark.parametrize("kind", ["general", "viscous"])
def test_manufactured_inertial_flow_converges_forms_E_and_M(kind):
    """On a smooth inertial-only flow both the effective-viscosity form
    (Form E, used on the GPU) and the paper's printed M/N/S/R form (Form M,
    with R = dN/dphi sign-corrected) converge to the analytic RHS at order
    >= 0.9, and their difference shrinks at the same rate."""
    errE, errM, errEM, errV, hs = [], [], [], [], []
    L = 0.5
    for nl in (10, 20, 40):
        h = L / nl
        p = lpgen.default_params(h)
        p.wall_z = -100.0
        st0 = lpgen.lattice_column(nl, nl, nl, h, seed=21, params=p)
        pts = np.stack([st0.x, st0.y, st0.z], 1)
        U, V, acc, dVdt = _manufactured(pts, p, kind)
        st = _state_from_points(pts, u=U, V=V)
        r = _one(st, p, brute=False).evaluate(form_m=True)
        c = np.array([L / 2] * 3)
        inner = np.all(np.abs(pts - c) < 0.11, axis=1)
        assert np.all((r["flags"][inner] >> 1) == oracle.BR_INERTIAL)
        sc = np.max(np.abs(acc[inner] - np.array(p.g)))
        errE.append(np.max(np.abs(r["acc"][:, inner].T - acc[inner])) / sc)
        errM.append(np.max(np.abs(r["accM"][:, inner].T - acc[inner])) / sc)
        errEM.append(np.max(np.abs(r["accM"][:, inner] - r["acc"][:, inner])) / sc)
        errV.append(np.max(np.abs(r["dVdt"][inner] - dVdt[inner]))
                    / np.max(np.abs(dVdt[inner])))
        hs.append(h)

    def order(e):
        return np.polyfit(np.log(hs), np.log(e), 1)[0]

    assert errE[-1] < 0.1 and errM[-1] < 0.1 and errV[-1] < 0.05, (errE, errM, errV)
    assert order(errE) >= 0.9 and order(errM) >= 0.9, (errE, errM)
    assert order(errV) >= 1.8, errV
    if kind == "general":
        assert order(errEM) >= 0.9, errEM
    else:
        assert errEM[-1] < 0.02, errEM
