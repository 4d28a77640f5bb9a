"""The substep histogram of the diagnostics (accepted substeps per cell and
step, bit-length bins) against the oracle's per-cell substep counts, taken
one step at a time, on every kernel path."""
import numpy as np
import pytest

import emma_inputs as E
import oracle
from gpu_helpers import groups_for, run_gpu

BINS = 18


def hist_of(counts):
    """bin 0: no substep; bin k: 2^(k-1) <= n < 2^k; the last bin from 2^16."""
    h = np.zeros(BINS, np.int64)
    for n in np.asarray(counts).ravel():
        h[0 if n <= 0 else min(int(n).bit_length(), BINS - 1)] += 1
    return h


def _case(shape, G, seed):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-3)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    cells = rng.integers(0, V, 5).astype(np.int64)
    rates = 10 ** rng.uniform(47, 50, 5)
    return dict(N=N, F=F, x=x, T=T, n0=n0, cells=cells, rates=rates, dx=dx, c=c, dt=E.courant_dt(dx, c))


def test_hist_of_bins():
    assert list(hist_of([0, 1, 2, 3, 4, 7, 8, 65535, 65536, 10 ** 6])[:4]) == [1, 1, 2, 2]
    h = hist_of([0, 1, 2, 3, 4, 7, 8, 65535, 65536, 10 ** 6])
    assert h[4] == 1 and h[16] == 1 and h[17] == 2 and h.sum() == 10


@pytest.mark.gpu
@pytest.mark.parametrize("path", ["split", "fused", "reference"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_substep_histogram_matches_oracle(path, precision):
    # three steps of a 10 x 11 x 12 grid with five sources: cell-steps with
    # 1 to about 100 substeps (bins 1..7), some beyond the first pass's budget
    k = _case((10, 11, 12), 3, 21)
    g = groups_for(3)
    steps = 3
    state = (k["N"], k["F"], k["x"], k["T"])
    want = np.zeros(BINS, np.int64)
    for _ in range(steps):
        o = oracle.run(*state, k["n0"], k["cells"], k["rates"], dx=k["dx"], c_red=k["c"], dt=k["dt"],
                       n_steps=1, groups=g, return_substeps=True)
        state = o[:4]
        want += hist_of(o[5])
    assert np.count_nonzero(want) >= 5
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], dx=k["dx"], c_red=k["c"],
                  dt=k["dt"], n_steps=steps, groups=g, precision=precision, path=path)
    got = np.array(gpu[4]["substep_hist"], dtype=np.int64)
    print(f"{path} {precision}: gpu {got[:9]} oracle {want[:9]}", flush=True)
    # every cell counted once per step, whatever pass finished it
    assert got.sum() == k["n0"].size * steps
    if precision == "fp64":
        assert np.array_equal(got, want)
        # consistent with the substep total: each bin's counts lie in its range
        lo = sum(int(got[b]) * (1 << (b - 1)) for b in range(1, BINS))
        assert lo <= gpu[4]["substeps"]
