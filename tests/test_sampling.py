"""The block sampling used by the full-size GPU tests, checked on the oracle
alone: k steps of the oracle on the (2r+1)^3 block around a cell (r > k)
give that cell bit for bit as the run on the whole periodic grid does, with
the block straddling the grid's faces and sources inside and outside it; a
cell more than k hops from every source evolves as the cell alone."""
import numpy as np

import emma_inputs as E
import oracle
from sampling import block, coords, hops_to_sources


def _groups(G):
    return oracle.group_constants(E.T_BB, E.EDGES[G])


def test_block_run_reproduces_full_grid_cells():
    w = E.make_workload("throughput256", n=24)
    rng = np.random.default_rng(5)
    w["src_cell"] = rng.integers(0, 24 ** 3, 12).astype(np.int64)
    w["src_cell"][3] = w["src_cell"][2]
    w["src_rate"] = 10 ** rng.uniform(48, 50, 12)
    steps = 4
    g = _groups(3)
    kw = dict(dx=w["dx"], c_red=w["c_red"], dt=w["dt"], n_steps=steps, groups=g)
    N, F, x, T, _ = oracle.run(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"], **kw)
    r = steps + 1
    cells = np.concatenate([w["src_cell"][:4], [0, 24 ** 3 - 1], rng.integers(0, 24 ** 3, 4)])
    lit = 0
    for cell in cells:
        cz, cy, cx = (int(v) for v in coords(np.int64(cell), w["shape"]))
        bN, bF, bx, bT, bn0, bc, br = block(w, (cz, cy, cx), r)
        oN, oF, ox, oT, _ = oracle.run(bN, bF, bx, bT, bn0, bc, br, **kw)
        assert np.array_equal(oN[:, r, r, r], N[:, cz, cy, cx])
        assert np.array_equal(oF[:, :, r, r, r], F[:, :, cz, cy, cx])
        assert ox[r, r, r] == x[cz, cy, cx] and oT[r, r, r] == T[cz, cy, cx]
        lit += N[:, cz, cy, cx].max() > 0
    assert lit >= 4
    far = np.nonzero(hops_to_sources(np.arange(24 ** 3), w) > steps + 1)[0]
    assert far.size > 0 and N.reshape(3, -1)[:, far].max() == 0.0
    z, y, xx = coords(far[:3], w["shape"])
    for k in range(3):
        sl = (slice(z[k], z[k] + 1), slice(y[k], y[k] + 1), slice(xx[k], xx[k] + 1))
        _, _, ox, oT, _ = oracle.run(w["N"][(slice(None),) + sl], w["F"][(slice(None), slice(None)) + sl],
                                     w["x"][sl], w["T"][sl], w["n0"][sl], np.zeros(0, np.int64),
                                     np.zeros(0), **kw)
        assert ox[0, 0, 0] == x[z[k], y[k], xx[k]] and oT[0, 0, 0] == T[z[k], y[k], xx[k]]
