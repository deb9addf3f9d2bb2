"""Host logic of the measurement tooling (CPU only): the HBM-traffic summary
that bench.py reports as roofline.traffic, the source-hash gate on it, and the
counter summaries behind the committed rocprofv3 profiles.  Inputs are small
synthetic counter files in the layout rocprofv3 writes (one row per dispatch
and counter)."""
import csv
import importlib.util
import json
import os

import pytest

from paper_1108_5673_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL = "void pwa::k_table_fused<float, 4, 4, true>(char const*, long, long, int, int)"
COPY = "__amd_rocclr_copyBuffer"


def _write_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (name, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_summarize_scales_each_counter_by_the_copy(tmp_path):
    # the copy of 1 GiB reads as half its bytes on FETCH_SIZE (scale 2) and
    # exactly on WRITE_SIZE (scale 1); a small copy of torch's is ignored
    gib_kib = (1 << 30) / 1024
    fetch = [(KERNEL, "FETCH_SIZE", v) for v in (781250.0, 781260.0, 781240.0, 781250.0, 781255.0)]
    fetch += [(COPY, "FETCH_SIZE", gib_kib / 2)] * 3 + [(COPY, "FETCH_SIZE", 12.0)]
    write = [(KERNEL, "WRITE_SIZE", 88.0)] * 5
    write += [(COPY, "WRITE_SIZE", gib_kib)] * 3 + [(COPY, "WRITE_SIZE", 24.0)]
    fp, wp, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _write_csv(fp, fetch)
    _write_csv(wp, write)
    res = profiling.summarize(str(fp), str(wp), str(out))
    assert res["fetch_scale"] == pytest.approx(2.0, rel=1e-15)
    assert res["write_scale"] == pytest.approx(1.0, rel=1e-15)
    # medians of the kernel's dispatches, in bytes, times the scale
    assert res["fetch_bytes_per_launch"] == pytest.approx(781250.0 * 1024 * 2, rel=1e-15)
    assert res["write_bytes_per_launch"] == pytest.approx(88.0 * 1024, rel=1e-15)
    assert res["hbm_bytes_per_launch"] == pytest.approx(
        res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"], rel=1e-15)
    assert res["algorithmic_bytes_per_launch"] == 1_000_000 * 1600
    assert res["dispatches"] == {"fetch": 5, "write": 5}
    assert res["kernel_source_sha256"] == profiling.kernel_source_hash()
    assert json.loads(out.read_text()) == res


def test_summarize_needs_the_kernel(tmp_path):
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write_csv(fp, [(COPY, "FETCH_SIZE", 1.0)])
    _write_csv(wp, [(COPY, "WRITE_SIZE", 1.0)])
    with pytest.raises(SystemExit):
        profiling.summarize(str(fp), str(wp), str(tmp_path / "t.json"))


def test_bench_reports_traffic_only_for_the_current_sources(tmp_path, monkeypatch):
    bench = _bench_module()
    rec = {"hbm_bytes_per_launch": 1.6e9, "kernel_source_sha256": profiling.kernel_source_hash()}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.measured_traffic() == 1.6e9
    rec["kernel_source_sha256"] = "0" * 64          # counters taken on other sources
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.measured_traffic() is None


def test_committed_traffic_matches_the_sources():
    """The committed counter summary was taken on the streaming kernel's
    current sources, so that bench.py reports it."""
    with open(os.path.join(ROOT, "profiles", "table_fused_w20_n1m_traffic.json")) as f:
        t = json.load(f)
    assert t["kernel_source_sha256"] == profiling.kernel_source_hash()
    # fetched within 0.1 % of the algorithmic bytes, written at most 1 MB
    assert abs(t["fetch_bytes_per_launch"] / t["algorithmic_bytes_per_launch"] - 1) < 1e-3
    assert 0 < t["write_bytes_per_launch"] < 1 << 20


def test_counters_takes_medians_over_files(tmp_path):
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    _write_csv(a, [("k_amp_hessian<3>", "MfmaUtil", v) for v in (40.0, 50.0, 45.0)]
               + [("k_other", "MfmaUtil", 99.0)])
    _write_csv(b, [("k_amp_hessian<3>", "SQ_INSTS_MFMA", v) for v in (1.0, 3.0)])
    res = profiling.counters("k_amp_hessian", [str(a), str(b)], str(tmp_path / "o.json"))
    assert res["counters"] == {"MfmaUtil": 45.0, "SQ_INSTS_MFMA": 2.0}
    assert res["dispatches"] == {"MfmaUtil": 3, "SQ_INSTS_MFMA": 2}
    assert res["names"] == ["k_amp_hessian<3>"]


@pytest.mark.parametrize("name,bf16", [
    ("_ZN3pwa10k_amp_mfmaIDF16bLi3ELi2ELb1EEEvPKT_", True),
    ("_ZN3pwa10k_amp_mfmaIDF16_Li3ELi2ELb0EEEvPKT_", False),
    ("void pwa::k_amp_mfma<bool _Accum, int, ELi, EL, bool, E>(bool _Accum)", True),
    ("void pwa::k_amp_mfma<_Float16, 3, 2, false>(...)", False),
])
def test_busy_files_each_instance_under_its_type(name, bf16):
    assert profiling._is_bf16(name) == bf16


@pytest.mark.parametrize("bf16,counted", [(True, 6.509e6), (False, 7.011e6)])
def test_batched_mfma_flops_agree_with_the_instruction_counter(bf16, counted):
    """bench.py's issued matrix-core FLOPs of one batched pass (10^6 events,
    W = 20, K = 256, V in two parts) against the matrix-core instructions the
    hardware counted for that pass (SQ_INSTS_MFMA medians per dispatch in
    profiles/amp_mfma_w20_n1m_k256_busy.md): the pass issues per 16-event
    tile and 32 vectors 6 forward (5 for bf16, whose second V part's last
    K-step rides in the first part's padding) and 4 adjoint 32x32x16 MFMAs of
    32768 FLOP and 4 adjoint 16x16x32 MFMAs of 16384 FLOP."""
    bench = _bench_module()
    n, w, k = 1_000_000, 20, 256
    per_tile_col = {"32x32x16": (5 if bf16 else 6) + 4, "16x16x32": 4}
    tile_cols = (n // 16) * (k // 32)
    insts = tile_cols * sum(per_tile_col.values())
    # the counter reads 0.14-0.16 % more instructions than this count
    assert abs(insts / counted - 1) < 2e-3
    flops = tile_cols * (per_tile_col["32x32x16"] * 32768 + per_tile_col["16x16x32"] * 16384)
    assert bench.mfma_flops(n, w, k, 2, bf16=bf16) == flops
    assert bench.mfma_algorithmic_flops(n, w, k, 2) == 8 * n * w * k * 4
