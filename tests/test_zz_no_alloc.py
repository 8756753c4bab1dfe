"""The allocation-free entry point lp_step_noalloc (static device workspace,
no context) against the existing entry point it varies, lp_step on a fresh
context: two calls in a row, the second on a smaller input, each compared
with lp_step on the same input (permutation bit-exact; every state array
within the FP64 parity bar of the step's increment), and sizes beyond the
static workspace rejected before any work."""
import sys

import numpy as np
import pytest

from cases import CASES

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lp():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2206_14061_amd as lp_mod
    lp_mod._lib.load()
    return lp_mod


def _step_both(lp, wl, **cfg):
    import torch
    ref_ctx = lp.make_context(wl, **cfg)
    ref = lp.DeviceState.from_host(wl.state)
    rperm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    ref_ctx.lp_step(ref, wl.dt, rperm)
    ref_ctx.sync_status()
    got = lp.DeviceState.from_host(wl.state)
    gperm = torch.empty(wl.n, dtype=torch.int32, device="cuda")
    lp.lp_step_noalloc(wl.offsets, wl.params, got, wl.dt, gperm, **cfg)
    torch.cuda.synchronize()
    return (got.to_host(), gperm.cpu().numpy()), (ref.to_host(), rperm.cpu().numpy())


def _compare(lp, wl, got, ref):
    (g, gp), (r, rp) = got, ref
    assert np.array_equal(gp, rp)
    old = wl.state.take(rp)
    exact = True
    for k, (a, b, c) in enumerate(zip(g.arrays(), r.arrays(), old.arrays())):
        d = np.max(np.abs(a - b))
        inc = np.max(np.abs(b - c))
        assert d <= TOL * inc, (lp.DeviceState.NAMES[k], d, inc)
        exact = exact and d == 0.0
    return exact


def test_noalloc_step_matches_lp_step_on_two_calls(lp):
    first = CASES["column16_flow_ragged"]()
    second = CASES["periodic_xy"]()
    assert second.n < first.n
    for wl in (first, second):
        _log("noalloc step: case %s n=%d systems=%d" % (wl.name, wl.n, wl.n_sys))
        got, ref = _step_both(lp, wl)
        exact = _compare(lp, wl, got, ref)
        _log("  matches lp_step (bitwise: %s)" % exact)


def test_noalloc_step_ensemble_and_refined(lp):
    wl = CASES["ensemble_3"]()
    _log("noalloc step: ensemble n=%d systems=%d, refined FP32" % (wl.n, wl.n_sys))
    got, ref = _step_both(lp, wl, precision=lp.LP_FP32_REFINED)
    _compare(lp, wl, got, ref)


def test_noalloc_rejects_sizes_beyond_its_workspace(lp):
    import torch
    wl = CASES["column16"]()
    n = 16385
    st = lp.DeviceState([torch.zeros(n, dtype=torch.float64, device="cuda")
                         for _ in range(7)])
    with pytest.raises(lp.LPError) as e:
        lp.lp_step_noalloc([0, n], wl.params, st, wl.dt)
    assert e.value.status == 2
    with pytest.raises(lp.LPError) as e:
        lp.lp_step_noalloc([0] * 65 + [100], wl.params * 65, st, wl.dt)
    assert e.value.status == 2
