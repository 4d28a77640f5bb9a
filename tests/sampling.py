"""Sampling a large run cell by cell: the block of cells a cell depends on
after k steps (periodic wrap), with the sources inside it, and the
face-neighbour distance to the nearest source."""
import numpy as np


def coords(cell, shape):
    nz, ny, nx = shape
    return cell // (ny * nx), (cell // nx) % ny, cell % nx


def block(w, center, r):
    """The (2r+1)^3 block around ``center`` (periodic wrap) and the sources
    inside it, in list order, as block-local flat indices."""
    shape = w["shape"]
    cz, cy, cx = center
    idx = [np.arange(c - r, c + r + 1) % n for c, n in zip((cz, cy, cx), shape)]
    sel = np.ix_(*idx)
    b = 2 * r + 1
    N = w["N"][(slice(None),) + sel]
    F = w["F"][(slice(None), slice(None)) + sel]
    x, T, n0 = w["x"][sel], w["T"][sel], w["n0"][sel]
    sz, sy, sx = coords(w["src_cell"], shape)
    oz = (sz - (cz - r)) % shape[0]
    oy = (sy - (cy - r)) % shape[1]
    ox = (sx - (cx - r)) % shape[2]
    inside = (oz < b) & (oy < b) & (ox < b)
    cells = ((oz * b + oy) * b + ox)[inside].astype(np.int64)
    rates = w["src_rate"][inside]
    return N, F, x, T, n0, cells, rates


def hops_to_sources(cells, w):
    """Periodic face-neighbour distance (L1) from each cell to its nearest source."""
    shape = w["shape"]
    c = np.stack(coords(cells, shape), axis=1)[:, None, :]
    s = np.stack(coords(w["src_cell"], shape), axis=1)[None, :, :]
    n = np.array(shape)[None, None, :]
    d = np.abs(c - s)
    d = np.minimum(d, n - d)
    return d.sum(axis=2).min(axis=1)
