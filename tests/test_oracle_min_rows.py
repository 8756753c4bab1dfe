"""Pins of the oracle's minimum-real-rows reading (option min_real_rows):
a stencil with fewer real or mirror rows than the option (ghost rows not
counted) takes the linear fit of Sec. 3.1 step 7's first-order Taylor
columns, flagged; every other stencil keeps its quadratic fit unchanged.

- On the sparse random cloud (many stencils with a few neighbours and many
  ghost rows): the flagged set is exactly {stencil size < 9} plus the
  stencils the rank test already sent to the linear fit; their
  coefficients equal LAPACK's least-squares solve (numpy.linalg.lstsq) of
  the three linear Taylor columns of all their rows, ghosts included; the
  others are bit-identical with the option off.
"""
import numpy as np

import oracle
from cases import CASES


def _taylor_lin(e):
    return np.array([e[0], e[1], e[2]])


def test_min_real_rows_takes_linear_fit_on_few_real_rows():
    wl = CASES["sparse_cloud"]()
    st, p = wl.state, wl.params[0]
    rng = np.random.default_rng(17)
    f = rng.normal(size=st.n)
    o0 = oracle.Oracle(st, wl.offsets, wl.params)
    o9 = oracle.Oracle(st, wl.offsets, wl.params, dict(min_real_rows=9))
    nb = o9.neighbours()
    c0, fl0 = o0.fit(f[None, :], [1], [0])
    c9, fl9 = o9.fit(f[None, :], [1], [0])
    few = nb.sten_cnt < 9
    assert few.sum() > 100 and (~few).sum() > 100
    rows = nb.sten_cnt + np.array([bin(int(gm)).count("1") for gm in nb.ghost_mask])
    # stencils the rule changes: fewer than 9 real rows but 9 rows or more
    changed = few & (rows >= 9)
    assert changed.sum() > 50
    assert np.all(fl9[few] & oracle.FLAG_LINEAR)
    assert np.array_equal(fl9[~few], fl0[~few])
    assert np.array_equal(c9[:, :, ~few], c0[:, :, ~few])
    # the changed stencils: LAPACK on the linear columns of all rows
    pts = np.concatenate([np.stack([st.x, st.y, st.z], 1), nb.mirror_state[:3].T], 0)
    fa = np.concatenate([f, f[nb.mirror_src]])
    for i in np.nonzero(changed)[0][::3]:
        ids = nb.sten_idx[i, :nb.sten_cnt[i]]
        A = [_taylor_lin(e) for e in (pts[ids] - pts[i]) / p.h]
        b = list(fa[ids] - f[i])
        for q in range(8):
            if nb.ghost_mask[i] >> q & 1:
                A.append(np.array([1.0 if q & 1 else -1.0, 1.0 if q & 2 else -1.0,
                                   1.0 if q & 4 else -1.0]))
                b.append(0.0)
        want = np.linalg.lstsq(np.array(A), np.array(b), rcond=None)[0] / p.h
        assert np.max(np.abs(c9[0, :3, i] - want)) <= 1e-10 * np.max(np.abs(want))
        assert np.all(c9[0, 3:, i] == 0.0)
        # and it differs from the quadratic fit the option replaces (where
        # the rank test had kept that one)
        if not fl0[i] & oracle.FLAG_LINEAR:
            assert np.max(np.abs(c0[0, :, i] - c9[0, :, i])) > 0

