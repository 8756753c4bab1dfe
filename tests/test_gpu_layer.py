"""Granular-layer compression (Sec. 4.1): the 3D periodic layer stepped on
the GPU against the reduced 1D model of the oracle (oracle/layer1d.py,
pinned by its exact equilibria and its settled height).

Both start at rest with the same solid-fraction profile (mean 0.5) and
compact under gravity.  Height measure on both sides: twice the mass
centroid (particle masses proportional to the initial solid fraction on
the lattice; cell masses in 1D).  The two agree to a few 1e-3 while the
layer compacts and to 2% once it has settled (the 3D wall is the
method's mirror boundary, the 1D wall a fixed node)."""
import numpy as np
import pytest

import lpgen
from oracle import layer1d
from test_gpu_parity import _log, lp  # noqa: F401

pytestmark = pytest.mark.gpu


def _heights_1d(wl, t_end, every):
    p = wl.params[0]
    H0, N = 0.03, 40
    zc = (np.arange(N) + 0.5) * H0 / N
    s = layer1d.layer_from_profile(lpgen.layer_profile(zc, H0), H0 / N, p.rho_s)
    dt = 2e-6
    per = int(round(every / dt))
    out = []
    for k in range(int(round(t_end / dt)) + 1):
        if k % per == 0:
            c = 0.5 * (s.z[1:] + s.z[:-1])
            out.append(2.0 * float(np.sum(s.m * c) / np.sum(s.m)))
        layer1d.step(p, s, dt)
    return np.array(out)


def test_periodic_layer_compacts_like_the_1d_model(lp):
    import torch
    wl = lpgen.layer_periodic()
    every, t_end = 0.005, 0.05
    per = int(round(every / wl.dt))
    ctx = lp.make_context(wl)
    st = lp.DeviceState.from_host(wl.state)
    ids = torch.arange(wl.n, dtype=torch.int32, device="cuda")
    mass = torch.tensor(1.0 / wl.state.V, device="cuda")
    h3 = []
    for c in range(int(round(t_end / every)) + 1):
        if c:
            ctx.lp_step_graph(st, wl.dt, per, ids)
        ctx.sync_status()
        m = mass[ids.long()]
        h3.append(2.0 * float((st.t[2] * m).sum() / m.sum()))
    h3 = np.array(h3)
    h1 = _heights_1d(wl, t_end, every)
    for k, (a, b) in enumerate(zip(h3, h1)):
        _log("t %.3f  3D %.6f  1D %.6f  (%+.2e)" % (k * every, a, b, a / b - 1.0))
    assert np.all(np.abs(h3[:6] / h1[:6] - 1.0) <= 3e-3)      # t <= 0.025 s
    assert np.all(np.abs(h3[7:] / h1[7:] - 1.0) <= 2e-2)      # t >= 0.035 s
    assert h3[-1] < 0.88 * h3[0]                               # it did compact
