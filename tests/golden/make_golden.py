"""Writes the stored oracle values that the full-length GPU parity tests
compare against (run from the repository root:
``python tests/golden/make_golden.py [lognormal128|throughput256]``).

Only the serial FP64 oracle and the seeded input generators are called.  For
each workload the oracle advances the whole grid over all of its steps, in
calls of ``SEG`` steps, and at every checkpoint stores
  * every field (N and F per group, x, T) at a fixed set of sampled cells:
    the source cells, random cells, cells the radiation reached and cells on
    the ionisation fronts (chosen from the oracle's own end state);
  * the largest magnitude of each field over the whole grid (the denominator
    of the normwise errors).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import emma_inputs as E  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SEG = {"lognormal128": 20, "throughput256": 10}
N_RANDOM, N_LIT, N_FRONT, N_SRC = 768, 768, 384, 128


def pick_cells(w, N, x, seed):
    """Sampled cells (sorted, unique) from the end state of the oracle run."""
    rng = np.random.default_rng(seed)
    V = w["n0"].size
    src = np.unique(w["src_cell"])
    if src.size > N_SRC:
        src = np.sort(rng.choice(src, N_SRC, replace=False))
    rand = rng.choice(V, N_RANDOM, replace=False)
    lit = np.nonzero(N.sum(axis=0).reshape(-1) > 0)[0]
    lit = rng.choice(lit, min(N_LIT, lit.size), replace=False)
    xf = x.reshape(-1)
    front = np.nonzero((xf > 0.05) & (xf < 0.95))[0]
    front = rng.choice(front, min(N_FRONT, front.size), replace=False)
    return np.unique(np.concatenate([src, rand, lit, front])).astype(np.int64)


def make(name):
    w = E.make_workload(name)
    g = oracle.group_constants(w["T_bb"], w["edges"])
    G, steps, seg = w["G"], w["steps"], SEG[name]
    N, F, x, T = w["N"], w["F"], w["x"], w["T"]
    states = []
    t0 = time.perf_counter()
    for s in range(seg, steps + 1, seg):
        N, F, x, T, cnt = oracle.run(N, F, x, T, w["n0"], w["src_cell"], w["src_rate"], dx=w["dx"],
                                     c_red=w["c_red"], dt=w["dt"], n_steps=seg, groups=g)
        states.append((s, N.copy(), F.copy(), x.copy(), T.copy()))
        print(f"{name}: step {s}/{steps}, {time.perf_counter() - t0:.0f} s, counters {cnt}", flush=True)
    cells = pick_cells(w, N, x, seed=2024)
    out = {"cells": cells, "steps": np.array([s[0] for s in states], dtype=np.int64)}
    out["N"] = np.stack([s[1].reshape(G, -1)[:, cells] for s in states])
    out["F"] = np.stack([s[2].reshape(G, 3, -1)[:, :, cells] for s in states])
    out["x"] = np.stack([s[3].reshape(-1)[cells] for s in states])
    out["T"] = np.stack([s[4].reshape(-1)[cells] for s in states])
    out["N_max"] = np.stack([np.abs(s[1]).reshape(G, -1).max(axis=1) for s in states])
    out["F_max"] = np.stack([np.abs(s[2]).reshape(G, -1).max(axis=1) for s in states])
    out["x_max"] = np.array([np.abs(s[3]).max() for s in states])
    out["T_max"] = np.array([np.abs(s[4]).max() for s in states])
    path = os.path.join(HERE, f"{name}_oracle.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path}: {cells.size} cells x {len(states)} checkpoints", flush=True)


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["lognormal128", "throughput256"]):
        make(name)
