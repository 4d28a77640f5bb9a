"""Throughput of the M1 transport + thermochemistry step on one MI355X.

Workload (default): 256^3 periodic grid, 3 photon groups (13.6/24.6/54.4/1000 eV,
1e5 K black body), log-normal hydrogen density (sigma_ln = 1, mean 1e-3 cm^-3,
P(k) ~ k^-2, seed 3), 256 point sources at random cells with log-uniform rates
1e47-1e50 photons/s, c_red = 0.1 c, dt = 0.8 dx / (3 c_red), from a dark, cold
(100 K), nearly neutral (x = 1.2e-3) start.  A step is one pass of the whole
path: source table (once per call), transport of all groups, chemistry subcycle.

Prints ONE JSON line: cell-updates/s of the FP32-transport / FP64-chemistry
path (the metric: the median of `--reps` calls of `--steps` steps, each from a
fresh copy of the initial state, after `--warmup` untimed steps), the all-FP64
path on the same inputs, the roofline figure of the dominant kernel
(algorithmic bytes per launch over its average duration from HIP events in one
more call of the same steps), the substep histogram, and the CPU oracle timed
on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s


def algorithmic_bytes(kernel, G, elem):
    """Bytes a kernel must move per cell: each field read or written once.
    N, F: 4 G values of `elem` bytes; x, T, n0: doubles."""
    nf = 4 * G * elem
    if kernel == "transport":
        return 2 * nf
    if kernel in ("chemistry", "fused_step", "step"):
        return 2 * nf + 3 * 8 + 2 * 8
    # adjoint, per cell-step: the chemistry adjoint reads U* (before the floor
    # and limiter), x, T, n0, dL/dN, dL/dF, dL/dx, dL/dT and dL/dn0 and writes
    # dL/dU* (storage type), dL/dx, dL/dT and dL/dn0; the transport adjoint
    # reads N, F and dL/dU* and writes dL/dN, dL/dF
    if kernel == "adj_chemistry":
        return 3 * nf + 3 * 8 + 2 * 8 + 2 * 8 + 2 * 8
    if kernel == "adj_transport":
        return 3 * nf
    return None


def kernel_fracs(kern, G, elem, V):
    """Each timed kernel's algorithmic bytes per step over its own measured
    time per step, as a fraction of the HBM peak (transport: N, F in and out;
    chemistry and the fused step: the whole state in and out plus n0)."""
    out = {}
    for k, (n, ms) in kern.items():
        b = algorithmic_bytes(k, G, elem)
        if b is None or ms <= 0:
            continue
        out[k] = b * V / (ms / n * 1e-3) / HBM_PEAK
    return out


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1508_07888_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not f.endswith((".hip", ".hpp")):
            continue
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


COPY_BYTES = 1 << 30  # calibration copy: reads and writes 1 GiB


def copy_calibration():
    """A plain elementwise kernel of known traffic (1 GiB read, 1 GiB written),
    run so that a counter pass sees FETCH_SIZE / WRITE_SIZE of a kernel whose
    HBM bytes are known; the ratio scales the counters of the step kernels."""
    import torch
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    del a, b


def _kernel_rows(csv_path):
    import csv
    with open(csv_path) as fh:
        return list(csv.DictReader(fh))


def _kind(name, precision="mixed"):
    """Kernel kind and whether it is the diagnostics-free instantiation of the
    given precision's storage type (float: mixed, double: fp64)."""
    if "emma::" not in name or "<" not in name:
        return None, False
    targs = [t.strip() for t in name[name.index("<") + 1:name.index(">")].split(",")]
    storage = "float" if precision == "mixed" else "double"
    product = not (len(targs) > 2 and targs[2] == "true") and len(targs) > 1 and targs[1] == storage
    if "k_chem_adj_list<" in name:
        return "adj_chemistry_deferred", targs[1] == storage
    if "k_chem_adj<" in name:
        return "adj_chemistry", targs[1] == storage
    if "k_transport_adj<" in name:
        return "adj_transport", targs[0] == storage
    if "k_tiled_hll<" in name:  # <storage, DIAG, TY, FULL>
        return "transport", targs[0] == storage and targs[1] == "false"
    if "k_tiled<" in name:
        return ("fused_step" if targs[3] == "true" else "transport"), product
    if "k_step_cell<" in name:
        return "fused_step", product
    if "k_step_ws<" in name:
        return "fused_step", product
    if "k_chem<" in name:
        return "chemistry", product
    if "k_transport<" in name:
        return "transport", product
    return None, False


def summarize_pmc(fetch_dir, write_dir, workload, precision, out_dir, command):
    """HBM bytes per launch of the step kernels from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by the ratio
    of the known bytes of the calibration kernel to what the same counter
    reads for it."""
    import glob
    counters = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        per, calib = {}, []
        for r in _kernel_rows(f):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"]) * 1024.0
            kind, product = _kind(r["Kernel_Name"], precision)
            if kind and product:
                per.setdefault(kind, []).append(v)
            elif "MulFunctor" in r["Kernel_Name"] and v > COPY_BYTES / 4:
                calib.append(v)  # the calibration kernel: torch.mul over 1 GiB
        if not calib:
            raise RuntimeError(f"no calibration kernel found in {f}")
        counters[counter] = (COPY_BYTES / max(calib), max(calib), {k: sum(v) / len(v) for k, v in per.items()})
    written = []
    for kind in counters["FETCH_SIZE"][2]:
        ff, fc, fk = counters["FETCH_SIZE"]
        wf, wc, wk = counters["WRITE_SIZE"]
        if kind not in wk:
            continue
        d = {"kernel": kind, "workload": workload, "precision": precision, "source_hash": source_hash(),
             "fetch_kib_raw": fk[kind] / 1024, "write_kib_raw": wk[kind] / 1024,
             "calibration": {"bytes_each_way": COPY_BYTES, "fetch_reads_bytes": fc, "write_reads_bytes": wc,
                             "fetch_factor": ff, "write_factor": wf},
             "fetch_bytes_per_launch": fk[kind] * ff, "write_bytes_per_launch": wk[kind] * wf,
             "hbm_bytes_per_launch": fk[kind] * ff + wk[kind] * wf, "commands": command}
        path = os.path.join(out_dir, f"{kind}_{workload}_{precision}_pmc.json")
        with open(path, "w") as fh:
            json.dump(d, fh, indent=1)
        written.append(path)
    return written


def summarize_sq(sq_dir, out_path, command):
    """Short text summary of a rocprofv3 --pmc run of SQ counters: per kernel,
    the mean per dispatch and the VALU / memory instructions per wave."""
    import glob
    f = glob.glob(os.path.join(sq_dir, "**", "*counter_collection.csv"), recursive=True)[0]
    agg = {}
    for r in _kernel_rows(f):
        kind, product = _kind(r["Kernel_Name"])
        if not kind:
            continue
        name = r["Kernel_Name"].split("(")[0].replace("|", "/")
        agg.setdefault(name, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    lines = ["# rocprofv3 SQ counters (mean per dispatch)", "", f"command: `{command}`", "",
             "| kernel | waves | VALU instr / wave | VMEM instr / wave | LDS instr / wave | wave cycles / wave |",
             "|---|---|---|---|---|---|"]
    for name, d in sorted(agg.items()):
        m = {c: sum(v) / len(v) for c, v in d.items()}
        w = max(m.get("SQ_WAVES", 0.0), 1.0)
        lines.append(f"| {name} | {m.get('SQ_WAVES', 0):.0f} | {m.get('SQ_INSTS_VALU', 0) / w:.1f} | "
                     f"{m.get('SQ_INSTS_VMEM', 0) / w:.1f} | {m.get('SQ_INSTS_LDS', 0) / w:.1f} | "
                     f"{m.get('SQ_WAVE_CYCLES', 0) / w:.0f} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    # machine-readable means per kernel, for the benchmark's VALU figures
    side = {"source_hash": source_hash(), "command": command,
            "kernels": {name: {c: sum(v) / len(v) for c, v in d.items()} for name, d in agg.items()}}
    with open(os.path.splitext(out_path)[0] + ".json", "w") as fh:
        json.dump(side, fh, indent=1)
    return out_path


def valu_from_profiles(kernel_prefix):
    """Per-wave VALU figures of one kernel instantiation from the committed SQ
    counter summary of the split path: instructions, VALU-active and
    resident cycles, and the share of a SIMD's issue slots its resident
    waves use (waves per SIMD x active / resident); None when there is no
    summary or the kernels changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "split_step_throughput256_sq_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != source_hash():
        return None
    for name, m in d["kernels"].items():
        if name.startswith(kernel_prefix):
            w = max(m.get("SQ_WAVES", 0.0), 1.0)
            act, cyc = m["SQ_ACTIVE_INST_VALU"] / w, m["SQ_WAVE_CYCLES"] / w
            return {"kernel": name, "valu_instr_per_wave": m["SQ_INSTS_VALU"] / w,
                    "valu_active_per_wave": act, "wave_cycles": cyc, "waves_per_simd": 4,
                    "simd_valu_busy": 4 * act / cyc}
    return None


# MI355X: 256 CUs x 4 SIMDs of 16 lanes at 2.4 GHz; a wave64 VALU instruction
# holds its SIMD for at least 4 cycles (FP64 FMA: 78.6 TFLOP/s in all).
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9


def valu_issue(cv, waves, avg_launch_s):
    """Share of the chip's VALU cycles over one launch (at the nominal clock)
    that the kernel's instructions (4 cycles each) and its measured
    VALU-active cycles (SQ_ACTIVE_INST_VALU, in units of 4 cycles) fill."""
    avail = avg_launch_s * SIMDS * CLOCK_HZ
    return {"valu_issue_frac": cv["valu_instr_per_wave"] * waves * 4 / avail,
            "valu_active_frac": cv["valu_active_per_wave"] * waves * 4 / avail}


def summarize_trace(trace_dir, out_path, command):
    """Short text summary of rocprofv3 --kernel-trace --stats (kernel stats CSV)."""
    import glob
    f = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = _kernel_rows(f)
    lines = ["# rocprofv3 kernel statistics", "", f"command: `{command}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|"]
    for r in rows:
        name = r["Name"].replace("|", "/")
        if len(name) > 110:
            name = name[:107] + "..."
        lines.append(f"| {name} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f}% |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return out_path


def substep_hist_labels(hist):
    """Cell-steps by accepted substeps, keyed by range: bit-length bins, "0",
    "1", "2-3", "4-7", ..., the last open-ended."""
    out = {}
    for b, n in enumerate(hist):
        if not n:
            continue
        if b == 0:
            key = "0"
        elif b == len(hist) - 1:
            key = f"{1 << (b - 1)}+"
        elif b == 1:
            key = "1"
        else:
            key = f"{1 << (b - 1)}-{(1 << b) - 1}"
        out[key] = n
    return out


def run_gpu(w, precision, steps, warmup, path="split", reps=5):
    import torch
    from paper_1508_07888_amd import EmmaRT
    dev = "cuda:0"
    G = w["G"]
    rt = EmmaRT(w["shape"], G, w["dx"], w["c_red"], precision=precision, T_bb=w["T_bb"],
                edges_eV=w["edges"], path=path, device=dev)
    fdt = rt.dtype
    N0 = torch.tensor(w["N"], dtype=fdt, device=dev)
    F0 = torch.tensor(w["F"], dtype=fdt, device=dev)
    x0 = torch.tensor(w["x"], dtype=torch.float64, device=dev)
    T0 = torch.tensor(w["T"], dtype=torch.float64, device=dev)
    n0 = torch.tensor(w["n0"], dtype=torch.float64, device=dev)
    cells = torch.tensor(w["src_cell"], dtype=torch.int64, device=dev)
    rates = torch.tensor(w["src_rate"], dtype=torch.float64, device=dev)
    N, F, x, T = N0.clone(), F0.clone(), x0.clone(), T0.clone()
    if warmup > 0:
        rt.step(N, F, x, T, n0, cells, rates, w["dt"], n_steps=warmup)
    # K steps from the initial state, inputs resident in HBM, once with HIP
    # events around every kernel (per-kernel durations for the roofline) ...
    N.copy_(N0); F.copy_(F0); x.copy_(x0); T.copy_(T0)
    rt.profile(True)
    rt.profile_read()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(rt.stream)
    rt.step(N, F, x, T, n0, cells, rates, w["dt"], n_steps=steps)
    stop.record(rt.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    kern = rt.profile_read()
    rt.profile(False)
    # ... then `reps` times without them, each from a fresh copy of the initial
    # state: the throughput is the median of these calls (min and max reported)
    rep_ms = []
    for _ in range(reps):
        N.copy_(N0); F.copy_(F0); x.copy_(x0); T.copy_(T0)
        torch.cuda.synchronize()
        start.record(rt.stream)
        rt.step(N, F, x, T, n0, cells, rates, w["dt"], n_steps=steps)
        stop.record(rt.stream)
        torch.cuda.synchronize()
        rep_ms.append(start.elapsed_time(stop) / steps)
    # untimed diagnostic pass over the same steps (substep statistics)
    N.copy_(N0); F.copy_(F0); x.copy_(x0); T.copy_(T0)
    d = rt.step(N, F, x, T, n0, cells, rates, w["dt"], n_steps=steps, diag=True,
                raise_on_status=False)
    torch.cuda.synchronize()
    rt.close()
    V = N0[0].numel()
    reps_out = None
    per_step = ms / steps
    if rep_ms:
        per_step = statistics.median(rep_ms)
        reps_out = {"count": len(rep_ms), "ms_per_step_median": per_step,
                    "ms_per_step_min": min(rep_ms), "ms_per_step_max": max(rep_ms),
                    "ms_per_step_with_kernel_events": ms / steps}
    return dict(value=V / (per_step * 1e-3), ms_per_step=per_step, kernels=kern,
                diag=d, V=V, elem=4 if precision == "mixed" else 8, reps=reps_out)


def run_variants(w, steps=10, reps=3):
    """The step's other kernel paths and options on the same inputs (mixed
    precision, `steps` steps from the initial state, median of `reps` calls
    after one warm-up step), next to the default split path over the same
    steps: the fused and reference paths, the HLL flux with M1 wave speeds
    (reference, split and fused paths), open boundaries with a planar inflow beam, the case-A
    chemistry with recombination photons, and static refinement (chemistry on
    the 2^3 children of the 4096 densest cells, emma_rt_step_crta)."""
    import numpy as np
    import torch
    from paper_1508_07888_amd import EmmaRT
    dev = "cuda:0"
    G, V = w["G"], w["n0"].size
    beam = float(w["c_red"] * 1e-6)  # inflow through z-: N = 1e-6 photons/cm^3 moving along +z
    cases = {
        "split": {},
        "fused": dict(path="fused"),
        "reference_glf": dict(path="reference"),
        "reference_hll": dict(path="reference", flux="hll"),
        "split_hll": dict(flux="hll"),
        "fused_hll": dict(path="fused", flux="hll"),
        "open_boundaries": dict(bc=["transmissive", "transmissive", "reflective", "reflective", "inflow",
                                    "transmissive"], inflow=[0, 0, 0, 0, beam, 0]),
        "case_a": dict(otsa=False),
        "refined_cells": {},
    }
    n0 = torch.tensor(w["n0"], dtype=torch.float64, device=dev)
    cells = torch.tensor(w["src_cell"], dtype=torch.int64, device=dev)
    rates = torch.tensor(w["src_rate"], dtype=torch.float64, device=dev)
    ref = np.sort(np.argsort(-w["n0"].ravel(), kind="stable")[:4096]).astype(np.int64)
    child = np.zeros(w["src_cell"].size, np.int32)
    out = {}
    for name, kw in cases.items():
        rt = EmmaRT(w["shape"], G, w["dx"], w["c_red"], precision="mixed", T_bb=w["T_bb"], edges_eV=w["edges"],
                    device=dev, **kw)
        N0 = torch.tensor(w["N"], dtype=rt.dtype, device=dev)
        F0 = torch.tensor(w["F"], dtype=rt.dtype, device=dev)
        x0 = torch.tensor(w["x"], dtype=torch.float64, device=dev)
        T0 = torch.tensor(w["T"], dtype=torch.float64, device=dev)
        N, F, x, T = N0.clone(), F0.clone(), x0.clone(), T0.clone()
        if name == "refined_cells":
            gref = torch.tensor(ref, dtype=torch.int64, device=dev)
            nf0 = n0.reshape(-1)[gref].unsqueeze(1).repeat(1, 8).contiguous()
            xf0 = x0.reshape(-1)[gref].unsqueeze(1).repeat(1, 8).contiguous()
            Tf0 = T0.reshape(-1)[gref].unsqueeze(1).repeat(1, 8).contiguous()
            xf, Tf = xf0.clone(), Tf0.clone()
            gch = torch.tensor(child, dtype=torch.int32, device=dev)

            def call(k):
                rt.step_crta(N, F, x, T, n0, cells, rates, w["dt"], gref, 2, xf, Tf, nf0, n_steps=k,
                             src_child=gch)

            def reset():
                N.copy_(N0); F.copy_(F0); x.copy_(x0); T.copy_(T0); xf.copy_(xf0); Tf.copy_(Tf0)
        else:
            def call(k):
                rt.step(N, F, x, T, n0, cells, rates, w["dt"], n_steps=k)

            def reset():
                N.copy_(N0); F.copy_(F0); x.copy_(x0); T.copy_(T0)
        call(1)
        ms = []
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        for _ in range(reps):
            reset()
            torch.cuda.synchronize()
            start.record(rt.stream)
            call(steps)
            stop.record(rt.stream)
            torch.cuda.synchronize()
            ms.append(start.elapsed_time(stop) / steps)
        rt.close()
        med = statistics.median(ms)
        out[name] = {"ms_per_step": med, "cell_updates_per_s": V / (med * 1e-3), "vs_split": None}
        del N0, F0, x0, T0, N, F, x, T
        torch.cuda.empty_cache()
    for name in out:
        out[name]["vs_split"] = out["split"]["ms_per_step"] / out[name]["ms_per_step"]
    out["steps"] = steps
    out["refined_cells"]["n_ref"] = int(ref.size)
    return out


def run_adjoint(w, precision, K=10, reps=3):
    """emma_rt_step_adjoint over K steps from the initial state (the segment's
    forward recomputed into the tape, then the reverse sweep), loss = sum of
    x_HII over the central 64^3 block: median of `reps` calls after one
    warm-up call, per step of the segment."""
    import torch
    from paper_1508_07888_amd import EmmaRT
    dev = "cuda:0"
    G = w["G"]
    rt = EmmaRT(w["shape"], G, w["dx"], w["c_red"], precision=precision, T_bb=w["T_bb"], edges_eV=w["edges"],
                adjoint_max_steps=K, device=dev)
    fdt = rt.dtype
    N0 = torch.tensor(w["N"], dtype=fdt, device=dev)
    F0 = torch.tensor(w["F"], dtype=fdt, device=dev)
    x0 = torch.tensor(w["x"], dtype=torch.float64, device=dev)
    T0 = torch.tensor(w["T"], dtype=torch.float64, device=dev)
    n0 = torch.tensor(w["n0"], dtype=torch.float64, device=dev)
    cells = torch.tensor(w["src_cell"], dtype=torch.int64, device=dev)
    rates = torch.tensor(w["src_rate"], dtype=torch.float64, device=dev)
    n = w["shape"][0]
    lo, hi = n // 2 - 32, n // 2 + 32
    gx0 = torch.zeros_like(x0)
    gx0[lo:hi, lo:hi, lo:hi] = 1.0
    gN, gF, gx, gT = torch.zeros_like(N0), torch.zeros_like(F0), gx0.clone(), torch.zeros_like(T0)
    g_n0, g_rate = torch.zeros_like(n0), torch.zeros_like(rates)

    def call():
        gN.zero_(); gF.zero_(); gx.copy_(gx0); gT.zero_(); g_n0.zero_(); g_rate.zero_()
        rt.step_adjoint(N0, F0, x0, T0, n0, cells, rates, w["dt"], K, gN, gF, gx, gT, g_n0, g_rate)

    call()
    rt.profile(True)
    rt.profile_read()
    call()
    torch.cuda.synchronize()
    kern = rt.profile_read()
    rt.profile(False)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(reps):
        torch.cuda.synchronize()
        start.record(rt.stream)
        call()
        stop.record(rt.stream)
        torch.cuda.synchronize()
        ms.append(start.elapsed_time(stop) / K)
    finite = bool(torch.isfinite(g_n0).all().item() and torch.isfinite(g_rate).all().item())
    rt.close()
    med = statistics.median(ms)
    V = w["n0"].size
    elem = 4 if precision == "mixed" else 8
    fracs = {}
    for k, (n, kms) in kern.items():
        b = algorithmic_bytes(k, G, elem) if k.startswith("adj_") else None
        if b is not None and kms > 0:
            fracs[k] = b * V * K / (kms * 1e-3) / HBM_PEAK
    return {"ms_per_step": med, "cell_steps_per_s": V / (med * 1e-3), "K": K,
            "scratch_GB": rt_scratch_gb(w, precision, K), "gradients_finite": finite,
            "kernels_ms_per_step": {k: v[1] / K for k, v in kern.items()}, "kernels_frac": fracs}


def rt_scratch_gb(w, precision, K):
    from paper_1508_07888_amd import _lib
    cfg = _lib.emma_rt_config()
    nz, ny, nx = w["shape"]
    cfg.nx, cfg.ny, cfg.nz, cfg.n_groups = nx, ny, nz, w["G"]
    cfg.dx, cfg.c_red = w["dx"], w["c_red"]
    cfg.precision = _lib.EMMA_RT_MIXED if precision == "mixed" else _lib.EMMA_RT_FP64
    cfg.otsa, cfg.max_substeps, cfg.adjoint_max_steps = 1, 100000, K
    for g in range(w["G"]):
        cfg.sigma_N[g] = cfg.sigma_E[g] = cfg.mean_E[g] = cfg.src_frac[g] = 1.0
    return _lib.emma_rt_scratch_bytes(cfg) / 1e9


# The CPU baseline: the serial FP64 oracle as it stands, one process per leg,
# each single-threaded.  Legs: the parity build (-O2 -ffp-contract=off) and a
# timing-only build (-O3 -march=native, compiled here for this host), each on
# the first steps of the benchmark's 256^3 inputs (truncated: the whole
# 50-step run is ~10 min per build) and on the whole 128^3, 100-step workload;
# then a replicated aggregate: one independent oracle process per usable core
# (at most 16) on the first steps of the 128^3 workload, summed.
CPU_LEGS = (("throughput256", 5, "O2"), ("throughput256", 5, "O3native"),
            ("lognormal128", 100, "O2"), ("lognormal128", 100, "O3native"))
REPLICATED_STEPS = 10


def cpu_leg(workload, steps, lib_path):
    """One leg, run in a child process: prints its JSON line."""
    import oracle
    if lib_path:
        oracle.use_library(lib_path)
    import emma_inputs as E
    w = E.make_workload(workload)
    g = oracle.group_constants(w["T_bb"], w["edges"])
    t = time.perf_counter()
    oracle.run(w["N"], w["F"], w["x"], w["T"], w["n0"], w["src_cell"], w["src_rate"],
               dx=w["dx"], c_red=w["c_red"], dt=w["dt"], n_steps=steps, groups=g)
    s = time.perf_counter() - t
    cu = w["n0"].size * steps
    print(json.dumps({"workload": workload, "steps": steps, "of_steps": w["steps"], "seconds": s,
                      "cell_updates_per_s": cu / s}), flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


class CpuBaseline:
    """Starts the CPU legs as child processes (they run while the GPU is
    timed: one core each), then collects them and runs the replicated leg."""

    def __init__(self, mode):
        import subprocess
        import tempfile
        from oracle import build as obuild
        self.mode = mode
        self.tmp = tempfile.mkdtemp(prefix="emma_oracle_")
        self.libs = {"O2": None}
        if mode == "full":
            self.libs["O3native"] = obuild.build_timing(os.path.join(self.tmp, "liboracle_o3native.so"))
            legs = CPU_LEGS
        else:
            legs = (("throughput256", 1, "O2"),)
        self.procs = []
        for wl, steps, build in legs:
            cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", wl, str(steps), self.libs[build] or ""]
            self.procs.append(((wl, steps, build), subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True)))

    def _collect(self, procs):
        out = {}
        for (wl, steps, build), p in procs:
            o, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"CPU leg {wl}/{steps}/{build} failed ({p.returncode})")
            out[(wl, steps, build)] = json.loads(o.strip().splitlines()[-1])
            print(f"cpu leg done: {wl} {steps} steps, {build}, {out[(wl, steps, build)]['seconds']:.1f} s",
                  file=sys.stderr, flush=True)
        return out

    def finish(self):
        import shutil
        import subprocess
        res = self._collect(self.procs)
        legs = {}
        for (wl, steps, build), r in res.items():
            trunc = r["steps"] < r["of_steps"]
            legs[f"{wl}_{build}"] = {
                "cell_updates_per_s": r["cell_updates_per_s"], "seconds": r["seconds"], "steps": r["steps"],
                "of_steps": r["of_steps"], "truncated": trunc,
                "build": "g++ -O2 -ffp-contract=off (parity build)" if build == "O2"
                         else "g++ -O3 -march=native (timing build)"}
        main = res[("throughput256", 5 if self.mode == "full" else 1, "O2")]
        cpus = os.cpu_count()
        try:
            usable = len(os.sched_getaffinity(0))
        except AttributeError:
            usable = cpus
        out = {"value": main["cell_updates_per_s"], "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
               "sample": f"first {main['steps']} of the {main['of_steps']} steps of the same 256^3 inputs "
                         f"(truncated), serial FP64 oracle, parity build (g++ -O2 -ffp-contract=off), "
                         f"{main['seconds']:.1f} s on one core",
               "cpu_model": _cpu_model(), "cpu_count": cpus, "usable_cores": usable, "legs": legs}
        if self.mode == "full":
            P = max(1, min(usable, 16))
            cmd = [sys.executable, os.path.abspath(__file__), "--cpu-leg", "lognormal128", str(REPLICATED_STEPS),
                   self.libs["O3native"]]
            t = time.perf_counter()
            procs = [(("lognormal128", REPLICATED_STEPS, f"rep{k}"),
                      subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True)) for k in range(P)]
            rep = self._collect(procs)
            wall = time.perf_counter() - t
            V = 128 ** 3
            out["replicated"] = {
                "processes": P, "aggregate_cell_updates_per_s": P * V * REPLICATED_STEPS / wall,
                "per_process_mean": statistics.mean(r["cell_updates_per_s"] for r in rep.values()),
                "wall_s": wall,
                "label": f"aggregate throughput of {P} independent serial oracle processes (timing build), "
                         f"each on the first {REPLICATED_STEPS} steps of the 128^3 workload: a replicated "
                         "figure, not a parallel code"}
        shutil.rmtree(self.tmp, ignore_errors=True)
        return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="throughput256")
    ap.add_argument("--n", type=int, default=None, help="override the grid size")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="same as --cpu-baseline none")
    ap.add_argument("--cpu-baseline", default="full", choices=["full", "quick", "none"],
                    help="full: parity and -O3 builds on the truncated 256^3 run and the whole 128^3 run, "
                         "plus the replicated aggregate; quick: one step of the 256^3 run, parity build")
    ap.add_argument("--cpu-leg", nargs=3, metavar=("WORKLOAD", "STEPS", "LIB"), help=argparse.SUPPRESS)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--variants", action="store_true",
                    help="also time the other paths and options (fused, reference, HLL, open boundaries, "
                         "case A, refined cells) over 10 steps of the same inputs")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time emma_rt_step_adjoint over 10 steps (mixed and FP64)")
    ap.add_argument("--reps", type=int, default=5,
                    help="further timed calls of the same steps from fresh copies (median, min, max)")
    ap.add_argument("--path", default="split", choices=["split", "fused", "reference"],
                    help="kernel path (all compute the same step; split is the default and the fastest)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (for scaling rocprofv3 byte counters)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/*_pmc.json from two rocprofv3 --pmc output dirs and exit")
    ap.add_argument("--summarize-sq", metavar="SQ_DIR",
                    help="write a text summary of a rocprofv3 --pmc SQ_* run to --summary-out and exit")
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR",
                    help="write a profiles/ text summary of a rocprofv3 --kernel-trace --stats dir and exit")
    ap.add_argument("--summary-out", default=None,
                    help="output file for --summarize-trace, output directory for --summarize-pmc")
    ap.add_argument("--command", default="", help="profiling command recorded in the summary")
    args = ap.parse_args()
    if args.cpu_leg:
        cpu_leg(args.cpu_leg[0], int(args.cpu_leg[1]), args.cpu_leg[2])
        return
    if args.summarize_pmc:
        out = summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.workload, "mixed",
                            args.summary_out or os.path.join(ROOT, "profiles"), args.command)
        print("\n".join(out))
        return
    if args.summarize_sq:
        print(summarize_sq(args.summarize_sq, args.summary_out, args.command))
        return
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace, args.summary_out, args.command))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the radiation step is built and timed on a "
              "single MI355X (no multi-GPU path in this build); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import emma_inputs as E
    w = E.make_workload(args.workload, n=args.n)
    G = w["G"]
    cpu_mode = "none" if args.no_cpu_baseline else args.cpu_baseline
    # the CPU legs run on their own cores while the GPU is timed
    cpu = CpuBaseline(cpu_mode) if cpu_mode != "none" else None
    if args.copy_calibration:
        copy_calibration()
    mixed = run_gpu(w, "mixed", args.steps, args.warmup, args.path, args.reps)
    fp64 = None if args.no_fp64 else run_gpu(w, "fp64", args.steps, args.warmup, args.path, args.reps)

    kern = mixed["kernels"]
    dom = max((k for k in kern if k != "src_table"), key=lambda k: kern[k][1])
    launches, total_ms = kern[dom]
    avg_s = total_ms / launches * 1e-3
    per_cell = algorithmic_bytes(dom, G, mixed["elem"])
    bytes_launch = per_cell * mixed["V"]
    achieved = bytes_launch / avg_s
    traffic = traffic_from_profiles(dom, args.workload, "mixed")
    # the whole step against the same roofline: cell-updates/s x algorithmic
    # bytes per cell-update (the state in and out once, n0 read) / peak
    step_bytes = algorithmic_bytes("step", G, mixed["elem"])
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": traffic, "kernel": dom,
                "bytes_per_cell": per_cell, "avg_launch_ms": avg_s * 1e3,
                "step_frac": mixed["value"] * step_bytes / HBM_PEAK,
                "step_achieved": mixed["value"] * step_bytes / 1e9, "step_bytes_per_cell": step_bytes,
                "kernels_frac": kernel_fracs(kern, G, mixed["elem"], mixed["V"])}
    # the SQ counter summary is of the default command (this workload, split path)
    chem_valu = None
    if args.workload == "throughput256" and args.path == "split":
        chem_valu = valu_from_profiles("void emma::k_chem<3, float, false, true, false>")
    if chem_valu is not None and "chemistry" in kern:
        n, ms = kern["chemistry"]
        chem_valu.update(valu_issue(chem_valu, mixed["V"] / 64, ms / n * 1e-3))
    out = {
        "metric": "M1+chem cell-updates/s at 256^3x3 groups (FP32 transport + FP64 chemistry)",
        "value": mixed["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": w["shape"][0], "groups": G,
                   "sources": int(w["src_cell"].size), "c_red_over_c": w["c_red"] / E.C_LIGHT,
                   "precision": "mixed", "path": args.path},
        "roofline": roofline,
        # what binds the dominant kernel besides HBM: its VALU issue (SQ counters)
        "chemistry_valu": chem_valu,
        "group_cell_updates_per_s": mixed["value"] * G,
        "kernels_ms": {k: v[1] / v[0] for k, v in kern.items()},
        "substeps_per_cell_step": mixed["diag"]["substeps"] / (mixed["V"] * args.steps),
        "attempts_per_cell_step": mixed["diag"]["attempts"] / (mixed["V"] * args.steps),
        "max_substeps_cell_step": mixed["diag"]["max_sub"],
        "substep_hist": substep_hist_labels(mixed["diag"]["substep_hist"]),
        "repetitions": mixed["reps"],
    }
    if fp64 is not None:
        k64 = fp64["kernels"]
        dom64 = max((k for k in k64 if k != "src_table"), key=lambda k: k64[k][1])
        b64 = algorithmic_bytes(dom64, G, 8) * fp64["V"]
        a64 = b64 / (k64[dom64][1] / k64[dom64][0] * 1e-3)
        sb64 = algorithmic_bytes("step", G, 8)
        out["fp64"] = {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"], "repetitions": fp64["reps"],
                       "dtype": "f64", "kernel": dom64, "achieved_GBs": a64 / 1e9,
                       "frac": a64 / HBM_PEAK, "step_frac": fp64["value"] * sb64 / HBM_PEAK,
                       "step_bytes_per_cell": sb64, "kernels_frac": kernel_fracs(k64, G, 8, fp64["V"]),
                       "kernels_ms": {k: v[1] / v[0] for k, v in k64.items()}}
        out["mixed_over_fp64"] = mixed["value"] / fp64["value"]
    if args.variants:
        out["variants"] = run_variants(w)
    if args.adjoint:
        out["adjoint"] = {p: run_adjoint(w, p) for p in (("mixed",) if args.no_fp64 else ("mixed", "fp64"))}
    if cpu is not None:
        out["cpu_baseline"] = cpu.finish()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
