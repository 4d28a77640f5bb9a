"""emma_rt_step_noalloc (the library's fixed scratch, no device allocation)
against emma_rt_step (a context's own scratch) through the C ABI.

Both run the same kernels in the same order on the same inputs, so the end
states must agree bit for bit.  Two calls in a row, the second with a smaller
grid, fewer groups and another path, check that a call does not depend on
what the previous call left in the shared array (source mask, counters,
work list); a third repeats the first case after them.
"""
import numpy as np
import pytest
import torch

import emma_inputs as E
from gpu_helpers import DEV, groups_for, to_dev
from paper_1508_07888_amd import EmmaRT, _lib

pytestmark = pytest.mark.gpu

# (shape, G, precision, path, n_steps, seed, n_src)
CASES = [((44, 36, 70), 3, "mixed", "split", 3, 11, 9),
         ((20, 17, 24), 2, "fp64", "fused", 3, 12, 4),
         ((44, 36, 70), 3, "mixed", "split", 3, 11, 9)]


def _inputs(shape, G, seed, n_src):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / shape[2]
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-3)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    cells = rng.integers(0, V, n_src).astype(np.int64)
    cells[1] = cells[0]  # two sources in one cell
    rates = 10.0 ** rng.uniform(48, 50, n_src)
    return dict(N=N, F=F, x=x, T=T, n0=n0, cells=cells, rates=rates, c=c, dx=dx, dt=E.courant_dt(dx, c))


def _run(rt, w, steps, noalloc):
    fdt = rt.dtype
    N, F = to_dev(w["N"], fdt), to_dev(w["F"], fdt)
    x, T, n0 = to_dev(w["x"]), to_dev(w["T"]), to_dev(w["n0"])
    cells, rates = to_dev(w["cells"], torch.int64), to_dev(w["rates"])
    if noalloc:
        rc = rt.step_noalloc(N, F, x, T, n0, cells, rates, w["dt"], n_steps=steps)
    else:
        rc = rt.step(N, F, x, T, n0, cells, rates, w["dt"], n_steps=steps)
    torch.cuda.synchronize()
    assert rc == _lib.EMMA_RT_OK
    return [a.cpu() for a in (N, F, x, T)]


def test_noalloc_matches_step_on_consecutive_calls():
    for k, (shape, G, prec, path, steps, seed, n_src) in enumerate(CASES):
        print(f"noalloc case {k}: shape {shape} G={G} {prec} {path} steps={steps}", flush=True)
        w = _inputs(shape, G, seed, n_src)
        rt = EmmaRT(shape, G, w["dx"], w["c"], precision=prec, groups=groups_for(G), path=path, device=DEV)
        ref = _run(rt, w, steps, noalloc=False)
        got = _run(rt, w, steps, noalloc=True)
        rt.close()
        for name, a, b in zip(("N", "F", "x", "T"), got, ref):
            assert torch.equal(a, b), f"case {k}: {name} differs (max {float((a - b).abs().max()):.3e})"
        # the step did something: radiation moved and the gas responded
        assert not torch.equal(ref[2], torch.tensor(w["x"]))


def test_noalloc_rejects_a_grid_beyond_its_scratch():
    shape, G = (160, 160, 160), 3
    w = _inputs((4, 4, 4), G, 13, 2)
    rt = EmmaRT(shape, G, 6.6 * E.KPC / 160, w["c"], precision="mixed", groups=groups_for(G), device=DEV)
    N, F, x, T = rt.new_state()
    n0 = torch.full(shape, 1e-3, dtype=torch.float64, device=DEV)
    cells = torch.zeros(0, dtype=torch.int64, device=DEV)
    rates = torch.zeros(0, dtype=torch.float64, device=DEV)
    x0 = x.clone()
    rc = rt.step_noalloc(N, F, x, T, n0, cells, rates, E.courant_dt(rt.dx, rt.c_red), n_steps=1,
                         raise_on_status=False)
    torch.cuda.synchronize()
    rt.close()
    assert rc == _lib.EMMA_RT_EINVAL
    assert "scratch" in _lib.emma_rt_last_error(None)
    assert torch.equal(x, x0)  # nothing ran
