"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (normwise per field and group, max |gpu - oracle| / max |oracle|):
  FP64 path:  1e-12 on N, F, x_HII, T.
  Mixed path (float32 transport, float64 chemistry): 1e-4 on N and F,
  1e-6 absolute on x_HII; T is reported (and held to 1e-3).
"""
import numpy as np
import pytest
import torch

import emma_inputs as E
import oracle
from gpu_helpers import groups_for, normwise, run_gpu, to_dev, DEV

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _compare(gpu, ora, precision, label=""):
    gN, gF, gx, gT = gpu[:4]
    oN, oF, ox, oT = ora[:4]
    G = oN.shape[0]
    eN = normwise(gN, oN, True)
    eF = normwise(gF, oF, True)
    ex = float(np.max(np.abs(gx - ox)))
    eT = normwise(gT, oT)
    print(f"{label} {precision}: N {eN} F {eF} x(abs) {ex:.3e} T {eT:.3e}", flush=True)
    if precision == "fp64":
        assert max(eN) <= TOL64 and max(eF) <= TOL64
        assert normwise(gx, ox) <= TOL64 and eT <= TOL64
    else:
        assert max(eN) <= 1e-4 and max(eF) <= 1e-4
        assert ex <= 1e-6
        assert eT <= 1e-3


def _random_case(shape, G, seed, n_src=5):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-3)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    cells = rng.integers(0, V, n_src).astype(np.int64)
    if n_src > 2:
        cells[1] = cells[0]  # two sources share a cell
    rates = 10 ** rng.uniform(47, 50, n_src)
    return dict(N=N, F=F, x=x, T=T, n0=n0, cells=cells, rates=rates, dx=dx, c=c, dt=dt)


PATHS = ["fused", "split", "reference"]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,G,seed", [((7, 9, 11), 1, 1), ((16, 5, 33), 2, 2),
                                          ((12, 12, 12), 3, 3), ((3, 20, 70), 4, 4),
                                          ((1, 1, 1), 3, 5), ((1, 4, 64), 2, 6),
                                          ((9, 13, 130), 3, 7), ((40, 6, 66), 2, 8)])
def test_random_grids_match_oracle(precision, shape, G, seed, path):
    # ragged shapes: partial 64 x 4 tiles, z-chunks with a remainder, grids
    # thinner than the stencil (periodic self-neighbours)
    k = _random_case(shape, G, seed)
    g = groups_for(G)
    steps = 3
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=steps, groups=g)
    ora = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"],
                  precision=precision, path=path, **kw)
    _compare(gpu, ora, precision, f"{shape} G={G} {path}")
    if precision == "fp64":
        d, oc = gpu[4], ora[4]
        assert d["substeps"] == oc["substeps"] and d["attempts"] == oc["attempts"]
        assert d["max_sub"] == oc["max_sub"]
        assert d["neg_clamps"] == oc["neg_clamp"]
        if shape == (1, 1, 1):
            # every neighbour is the cell itself: the update returns U plus a
            # sum that cancels exactly in real arithmetic, so at the f = 1
            # cells of the input whether |F*| exceeds c N* is decided by the
            # last bit of the rounding (a legitimate decision flip); the
            # fields above agree to 1e-12 either way
            assert abs(d["limiter_hits"] - oc["limiter"]) <= G * steps
        else:
            assert d["limiter_hits"] == oc["limiter"]


@pytest.mark.parametrize("otsa,iso", [(0, 0), (1, 1), (0, 1)])
def test_chemistry_modes_match_oracle(otsa, iso):
    k = _random_case((10, 11, 12), 3, 9)
    g = groups_for(3)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=2, groups=g, otsa=otsa, isothermal=iso)
    ora = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    _compare(gpu, ora, "fp64", f"otsa={otsa} iso={iso}")


def test_substep_guard_matches_oracle_and_reports():
    k = _random_case((8, 8, 8), 2, 10)
    k["N"] *= 1e3
    g = groups_for(2)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=1, groups=g, max_substeps=2)
    ora = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    _compare(gpu, ora, "fp64", "cap")
    assert ora[4]["cap_hits"] > 0
    assert gpu[4]["cap_hits"] == ora[4]["cap_hits"]
    assert gpu[4]["status"] == -4  # ESUBSTEP


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_stromgren32_workload_200_steps(precision):
    # 32^3, one group, uniform gas, one 5e48 /s source at the centre, c_red = c.
    w = E.make_workload("stromgren32")
    g = groups_for(1)
    kw = dict(dx=w["dx"], c_red=w["c_red"], dt=w["dt"], n_steps=w["steps"], groups=g)
    ora = oracle.run(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"], **kw)
    gpu = run_gpu(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"],
                  precision=precision, **kw)
    _compare(gpu, ora, precision, "stromgren32")
    d = gpu[4]
    vol = w["dx"] ** 3
    emitted = w["src_rate"].sum() * w["steps"] * w["dt"]
    assert d["ionised"] - 1.2e-3 * 1e-3 * w["n0"].size * vol <= emitted * (1 + 1e-6)
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert abs(d["photons"][0] - ora[0].sum() * vol) <= tol * d["photons"][0]


def test_adjoint64_workload_forward_matches_oracle():
    # 64^3, two groups, log-normal gas (sigma_ln 0.8), 8 sources, 60 steps, FP64.
    w = E.make_workload("adjoint64")
    g = groups_for(2)
    kw = dict(dx=w["dx"], c_red=w["c_red"], dt=w["dt"], n_steps=w["steps"], groups=g)
    ora = oracle.run(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"], **kw)
    gpu = run_gpu(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"], **kw)
    _compare(gpu, ora, "fp64", "adjoint64")


def test_lognormal128_workload_mixed_first_steps():
    # Full 128^3 grid, three groups, 16 sources at density peaks; the oracle runs
    # the first 6 of the 100 steps (the rest is covered by the invariants test).
    w = E.make_workload("lognormal128")
    g = groups_for(3)
    kw = dict(dx=w["dx"], c_red=w["c_red"], dt=w["dt"], n_steps=6, groups=g)
    ora = oracle.run(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"], **kw)
    for precision in ("mixed", "fp64"):
        gpu = run_gpu(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"],
                      precision=precision, **kw)
        _compare(gpu, ora, precision, "lognormal128")


def test_zero_steps_and_no_sources():
    k = _random_case((6, 7, 8), 2, 11)
    g = groups_for(2)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], groups=g)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], n_steps=0, **kw)
    assert np.array_equal(gpu[0], k["N"]) and np.array_equal(gpu[2], k["x"])
    e = np.zeros(0, np.int64), np.zeros(0)
    ora = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], *e, n_steps=2, **kw)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], *e, n_steps=2, **kw)
    _compare(gpu, ora, "fp64", "no sources")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape", [(20, 12, 70), (33, 8, 64)])
def test_fused_and_split_paths_agree(precision, shape):
    # Same closure, flux and chemistry code in both; the two tilings may
    # round a product-plus-sum differently (the compiler fuses multiply-adds
    # where the surrounding code allows), so they agree to the parity
    # tolerances, not bit for bit.  Ragged and whole tiles.
    k = _random_case(shape, 3, 13)
    g = groups_for(3)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=5, groups=g, precision=precision)
    a = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], path="fused", **kw)
    b = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], path="split", **kw)
    errs = [normwise(u, v) for u, v in zip(a[:4], b[:4])]
    print(f"{shape} {precision}: max |fused - split| / max |split| (N, F, x, T) = {errs}", flush=True)
    tol = [1e-12] * 4 if precision == "fp64" else [1e-5, 1e-5, 1e-7, 1e-5]
    for e, t in zip(errs, tol):
        assert e <= t
    assert a[4]["limiter_hits"] == b[4]["limiter_hits"] and a[4]["neg_clamps"] == b[4]["neg_clamps"]
    assert abs(a[4]["substeps"] - b[4]["substeps"]) <= 1e-3 * b[4]["substeps"]


def test_runs_are_bitwise_reproducible():
    k = _random_case((9, 10, 11), 3, 12)
    g = groups_for(3)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=4, groups=g)
    for precision in ("fp64", "mixed"):
        for path in PATHS:
            a = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"],
                        precision=precision, path=path, **kw)
            b = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"],
                        precision=precision, path=path, **kw)
            for u, v in zip(a[:4], b[:4]):
                assert np.array_equal(u, v)


def test_host_errors_on_device():
    from paper_1508_07888_amd import EmmaRT, _lib
    n = 8
    rt = EmmaRT((n, n, n), 1, 1e20, 3e9, precision="fp64", groups=groups_for(1), device=DEV)
    N, F, x, T = rt.new_state()
    n0 = torch.full((n, n, n), 1e-3, dtype=torch.float64, device=DEV)
    cells = torch.tensor([3], dtype=torch.int64, device=DEV)
    rates = torch.tensor([1e48], dtype=torch.float64, device=DEV)
    with pytest.raises(_lib.EmmaError) as e:
        rt.step(N, F, x, T, n0, cells, rates, dt=1.01 * rt.max_dt())
    assert e.value.status == _lib.EMMA_RT_EINVAL
    with pytest.raises(_lib.EmmaError):
        rt.step(N, F, x, T, n0, cells, rates, dt=-1.0)
    with pytest.raises(_lib.EmmaError):
        rt.step(N, F, x, T, n0, cells, rates, dt=rt.max_dt(), n_steps=-1)
    # a source cell outside the grid is ignored and reported (never written)
    bad = torch.tensor([n ** 3 + 5], dtype=torch.int64, device=DEV)
    d = rt.step(N, F, x, T, n0, bad, rates, dt=rt.max_dt(), diag=True, raise_on_status=False)
    assert d["status"] == _lib.EMMA_RT_EINVAL
    # NaN in the input state is detected by the diagnostics
    T[1, 2, 3] = float("nan")
    d = rt.step(N, F, x, T, n0, cells, rates, dt=rt.max_dt(), diag=True, raise_on_status=False)
    assert d["status"] == _lib.EMMA_RT_ENONFINITE and d["nonfinite"] >= 1
    # the context stays usable after every error
    T.fill_(100.0)
    d = rt.step(N, F, x, T, n0, cells, rates, dt=rt.max_dt(), diag=True)
    assert d["status"] == 0
    rt.close()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("precision,scale,check", [("mixed", 1e-24, True), ("mixed", 1e-27, False),
                                                   ("mixed", 1e-31, False), ("fp64", 1e-161, True)])
def test_tiny_fields_ahead_of_a_front_stay_finite(precision, scale, check, path):
    # Radiation fields many orders of magnitude below the source's, as ahead
    # of a diffusive front, with |F|^2 near or below the smallest normal
    # number of the storage precision: the closure must neither overflow nor
    # produce NaN (regression: bq = (3 chi - 1)/2 N / |F|^2 overflowed).
    k = _random_case((20, 11, 12), 2, 31, n_src=0)
    N, F = k["N"] * scale, k["F"] * scale
    N[:, :5] = k["N"][:, :5]  # a lit slab next to the tiny region
    F[:, :, :5] = k["F"][:, :, :5]
    g = groups_for(2)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=3, groups=g)
    ora = oracle.run(N, F, k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    gpu = run_gpu(N, F, k["x"], k["T"], k["n0"], k["cells"], k["rates"], precision=precision, path=path, **kw)
    for a in gpu[:4]:
        assert np.all(np.isfinite(a))
    assert gpu[4]["nonfinite"] == 0
    _compare(gpu, ora, precision, f"tiny {scale:g} {path}")
    if check:
        # the planes the lit slab has not reached, relative to their own scale
        # (the storage precision still resolves |F|^2 there)
        sl = (slice(None), slice(8, 17))
        e = np.max(np.abs(gpu[0][sl] - ora[0][sl])) / np.max(np.abs(ora[0][sl]))
        print(f"tiny region N: {e:.2e}", flush=True)
        assert e <= (1e-12 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("n_src", [257, 3000])
def test_long_source_lists(n_src):
    # many sources (several 256-entry sorting tiles), most cells hosting
    # several of them, plus entries outside the grid: the sums per cell are in
    # list order as in the oracle, the outside entries are ignored (and
    # reported as EINVAL with diagnostics)
    shape, G = (10, 12, 14), 2
    k = _random_case(shape, G, 21, n_src=n_src)
    V = int(np.prod(shape))
    rng = np.random.default_rng(22)
    bad = rng.choice(n_src, 7, replace=False)
    cells = k["cells"].copy()
    cells[bad[:4]] = V + rng.integers(0, 1000, 4)
    cells[bad[4:]] = -1 - rng.integers(0, 1000, 3)
    ok = np.ones(n_src, bool)
    ok[bad] = False
    g = groups_for(G)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=2, groups=g)
    ora = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], cells[ok], k["rates"][ok], **kw)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], cells, k["rates"], precision="fp64", **kw)
    _compare(gpu, ora, "fp64", f"{n_src} sources")
    assert gpu[4]["status"] == -1  # EINVAL: out-of-grid sources were ignored
