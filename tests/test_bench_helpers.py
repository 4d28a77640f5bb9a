"""Host-side helpers of bench.py: the substep-histogram labels, the kernel
classification of profiler rows, and the staleness check of the committed
counter summaries."""
import json

import bench


def test_substep_hist_labels_cover_the_bit_length_bins():
    h = [0] * 18
    h[1], h[2], h[4], h[17] = 5, 3, 2, 1
    assert bench.substep_hist_labels(h) == {"1": 5, "2-3": 3, "8-15": 2, "65536+": 1}
    h[0] = 7
    assert bench.substep_hist_labels(h)["0"] == 7


def test_kernel_kinds_select_the_product_instantiation_of_the_precision():
    chem = "void emma::k_chem<3, float, false, true>(float const*, ...)"
    assert bench._kind(chem) == ("chemistry", True)
    assert bench._kind(chem.replace("false, true", "true, true")) == ("chemistry", False)  # diagnostics
    assert bench._kind(chem.replace("float", "double")) == ("chemistry", False)
    assert bench._kind(chem.replace("float", "double"), "fp64") == ("chemistry", True)
    tiled = "void emma::k_tiled<1, float, false, false, false, 4, 4, true>(emma::TileArgs<float>)"
    assert bench._kind(tiled) == ("transport", True)
    # the split transport as launched now: one plane of prefetch, one LDS buffer
    one_buf = "void emma::k_tiled<1, float, false, false, false, 4, 1, true, 1>(emma::TileArgs<float>)"
    assert bench._kind(one_buf) == ("transport", True)
    assert bench._kind(one_buf.replace("float, false", "float, true", 1)) == ("transport", False)
    assert bench._kind(one_buf.replace("float", "double"), "fp64") == ("transport", True)
    fused = "void emma::k_tiled<3, float, false, true, true, 4, 0, true>(emma::TileArgs<float>)"
    assert bench._kind(fused) == ("fused_step", True)
    # the HLL tiled transport: <storage, DIAG, tile rows, whole tiles>
    hll = "void emma::k_tiled_hll<float, false, 4, true>(emma::TileArgs<float>)"
    assert bench._kind(hll) == ("transport", True)
    assert bench._kind(hll.replace("float, false", "float, true")) == ("transport", False)
    assert bench._kind(hll.replace("float", "double"), "fp64") == ("transport", True)
    assert bench._kind("void emma::k_step_cell<3, float, false, true>(float const*)") == ("fused_step", True)
    assert bench._kind("void at::native::vectorized_elementwise_kernel<4, ...>") == (None, False)


def test_committed_counter_summaries_follow_the_sources(tmp_path, monkeypatch):
    # a summary taken from other sources is ignored (traffic / VALU figures null)
    current = bench.source_hash()
    d = {"source_hash": "0" * 16, "hbm_bytes_per_launch": 1.0}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "chemistry_w_mixed_pmc.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: current)
    assert bench.traffic_from_profiles("chemistry", "w", "mixed") is None
    d["source_hash"] = current
    (prof / "chemistry_w_mixed_pmc.json").write_text(json.dumps(d))
    assert bench.traffic_from_profiles("chemistry", "w", "mixed") == 1.0
    assert bench.valu_from_profiles("void emma::k_chem<3") is None  # no SQ summary there


def test_valu_issue_fractions_against_a_hand_count():
    # one wave per SIMD, each issuing 2.4e6 instructions of 4 cycles over 4 ms
    # at 2.4 GHz fills all the SIMDs' cycles; the active count (units of 4
    # cycles) likewise
    cv = {"valu_instr_per_wave": 2.4e6, "valu_active_per_wave": 1.2e6}
    f = bench.valu_issue(cv, bench.SIMDS, 4e-3)
    assert abs(f["valu_issue_frac"] - 1.0) < 1e-12 and abs(f["valu_active_frac"] - 0.5) < 1e-12
