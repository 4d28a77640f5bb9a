"""Helpers shared by the GPU tests: run the HIP path from numpy inputs and
compare with the oracle normwise (max |a - b| / max |b| per field and group)."""
import numpy as np
import torch

import emma_inputs as E
import oracle
from paper_1508_07888_amd import EmmaRT

DEV = "cuda:0"


def to_dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def run_gpu(N, F, x, T, n0, cells, rates, *, dx, c_red, dt, n_steps, groups, precision="fp64",
            otsa=1, isothermal=0, max_substeps=100000, diag=True, rt=None, path="split", bc=None,
            inflow=None, flux="glf"):
    G = N.shape[0]
    own = rt is None
    if own:
        rt = EmmaRT(n0.shape, G, dx, c_red, precision=precision, groups=groups, otsa=otsa,
                    isothermal=isothermal, max_substeps=max_substeps, path=path, device=DEV,
                    bc=bc, inflow=inflow, flux=flux)
    fdt = rt.dtype
    gN, gF = to_dev(N, fdt), to_dev(F, fdt)
    gx, gT, gn = to_dev(x), to_dev(T), to_dev(n0)
    gc, gr = to_dev(cells, torch.int64), to_dev(rates)
    d = rt.step(gN, gF, gx, gT, gn, gc, gr, dt, n_steps=n_steps, diag=diag,
                raise_on_status=False)
    torch.cuda.synchronize()
    out = (gN.double().cpu().numpy(), gF.double().cpu().numpy(), gx.cpu().numpy(),
           gT.cpu().numpy(), d)
    if own:
        rt.close()
    return out


def normwise(a, b, axis_groups=None):
    """max |a-b| / max |b|, per leading index when axis_groups is given."""
    if axis_groups is None:
        den = np.max(np.abs(b))
        return float(np.max(np.abs(a - b)) / den) if den > 0 else float(np.max(np.abs(a - b)))
    return [normwise(a[g], b[g]) for g in range(a.shape[0])]


def groups_for(G):
    return oracle.group_constants(E.T_BB, E.EDGES[G])
