"""HBM traffic of the streaming kernel from hardware counters.

Two steps, each run under rocprofv3 with one counter (FETCH_SIZE in one run,
WRITE_SIZE in another):

    rocprofv3 --pmc FETCH_SIZE -d <dir> -o fetch --output-format csv -- \\
        python3 -m paper_1108_5673_amd.profiling run
    rocprofv3 --pmc WRITE_SIZE -d <dir> -o write --output-format csv -- \\
        python3 -m paper_1108_5673_amd.profiling run
    python3 -m paper_1108_5673_amd.profiling summarize <fetch csv> <write csv> <out.json>

`run` evaluates the 1M-event, 20-wave complex64 table a few times and then
copies a buffer of known size (1 GiB) device to device.  `summarize` scales
each counter of the streaming kernel by the ratio of the copy's known bytes
to what the same counter read for the copy, and writes the per-launch HBM
bytes with the hash of the kernel sources they were measured on.

Matrix-core use of the batched kernel (k_amp_mfma, 256 vectors over the
1M-event, 20-wave sample, bf16 then fp16 amplitudes), one rocprofv3 run per
counter set:

    rocprofv3 --pmc MfmaUtil VALUBusy -d <dir> -o derived --output-format csv -- \\
        python3 -m paper_1108_5673_amd.profiling run-batched
    rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_ACTIVE_INST_VALU SQ_INSTS_MFMA \\
        SQ_INSTS_VALU SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE -d <dir> -o raw \\
        --output-format csv -- python3 -m paper_1108_5673_amd.profiling run-batched
    python3 -m paper_1108_5673_amd.profiling busy <derived csv> <raw csv> <out.json>

The same counters for the FUMILI matrix kernel (k_amp_hessian, nll_grad_hess on
the 1M-event, 20-wave sample in the FP32 amplitude form):

    rocprofv3 --pmc ... -- python3 -m paper_1108_5673_amd.profiling run-hess
    python3 -m paper_1108_5673_amd.profiling counters k_amp_hessian <csv> ... <out.json>
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SOURCES = ["paper_1108_5673_amd/csrc/k_table.hip", "paper_1108_5673_amd/csrc/wave_ops.h",
                  "paper_1108_5673_amd/csrc/pwa_internal.h"]
COPY_BYTES = 1 << 30
STREAM_KERNEL = "k_table_fused"


def kernel_source_hash() -> str:
    """SHA-256 over the sources of the streaming kernel."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def run(evals: int = 5) -> None:
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import paper_1108_5673_amd as pwa
    from paper_1108_5673_amd import synth

    torch.cuda.init()
    s = synth.make_sample("w20_n1m")
    m = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), s.n_gen, form="table")
    for k in range(evals):
        m.nll_grad(s.points[k])
    torch.cuda.synchronize()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    m.close()
    print("profiling run done: %d evaluations, 3 copies of %d bytes" % (evals, COPY_BYTES),
          flush=True)


def run_batched(reps: int = 4) -> None:
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import paper_1108_5673_amd as pwa
    from paper_1108_5673_amd import synth

    torch.cuda.init()
    s = synth.make_sample("w20_n1m_k256")
    d32, mc32 = s.data.astype(np.complex64), s.mc.astype(np.complex64)
    for form in ("amplitude_bf16", "amplitude_fp16"):
        m = pwa.Model(d32, mc32, s.n_gen, form=form)
        for _ in range(reps):
            pwa.nll_batched([m], [s.points])
        torch.cuda.synchronize()
        m.close()
    print("profiling run done: %d batched passes of 256 vectors per form" % reps, flush=True)


def run_hess(reps: int = 4) -> None:
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    import paper_1108_5673_amd as pwa
    from paper_1108_5673_amd import synth

    torch.cuda.init()
    s = synth.make_sample("w20_n1m")
    m = pwa.Model(s.data.astype(np.complex64), s.mc.astype(np.complex64), s.n_gen,
                  form="amplitude")
    for k in range(reps):
        m.nll_grad_hess(s.points[k])
    torch.cuda.synchronize()
    m.close()
    print("profiling run done: %d NLL + gradient + FUMILI matrix calls" % reps, flush=True)


def _rows(path: str):
    with open(path) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, counter: str):
    """{kernel name: [value per dispatch]} for one counter (KiB)."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def _pick(d, needle: str):
    names = [n for n in d if needle in n]
    if not names:
        raise SystemExit("no dispatch of a kernel named like %r in %s" % (needle, sorted(d)))
    vals = [v for n in names for v in d[n]]
    return names, vals


def summarize(fetch_csv: str, write_csv: str, out_json: str) -> dict:
    f = _per_dispatch(_rows(fetch_csv), "FETCH_SIZE")
    w = _per_dispatch(_rows(write_csv), "WRITE_SIZE")
    kf_names, kf = _pick(f, STREAM_KERNEL)
    kw_names, kw = _pick(w, STREAM_KERNEL)
    copy_f = [v for n, vs in f.items() if "opy" in n for v in vs]
    copy_w = [v for n, vs in w.items() if "opy" in n for v in vs]
    # the copies are the largest dispatches of a copy kernel
    copy_f = sorted(copy_f)[-3:]
    copy_w = sorted(copy_w)[-3:]
    scale_f = COPY_BYTES / (1024.0 * statistics.median(copy_f))
    scale_w = COPY_BYTES / (1024.0 * statistics.median(copy_w))
    fetch_b = 1024.0 * statistics.median(kf) * scale_f
    write_b = 1024.0 * statistics.median(kw) * scale_w
    res = {
        "kernel": kf_names[0],
        "workload": "w20_n1m: 1M events x 20 waves, complex64 table with a real diagonal",
        "algorithmic_bytes_per_launch": 1_000_000 * 200 * 8,   # 1600 B per event
        "fetch_kib_raw": statistics.median(kf),
        "write_kib_raw": statistics.median(kw),
        "copy_fetch_kib_raw": statistics.median(copy_f),
        "copy_write_kib_raw": statistics.median(copy_w),
        "copy_bytes": COPY_BYTES,
        "fetch_scale": scale_f,
        "write_scale": scale_w,
        "fetch_bytes_per_launch": fetch_b,
        "write_bytes_per_launch": write_b,
        "hbm_bytes_per_launch": fetch_b + write_b,
        "dispatches": {"fetch": len(kf), "write": len(kw)},
        "kernel_source_sha256": kernel_source_hash(),
    }
    with open(out_json, "w") as fo:
        json.dump(res, fo, indent=1)
        fo.write("\n")
    return res


def _is_bf16(name: str) -> bool:
    """bf16 instance of a kernel template, by its demangled or mangled name
    (the Itanium mangling of __bf16 is DF16b, of _Float16 DF16_).  The kernel
    has only the two 16-bit instances, and some demanglers cannot read DF16b
    (they print neither type name), so everything not marked as _Float16 is
    the bf16 instance."""
    if "bf16" in name or "DF16b" in name:
        return True
    return not ("DF16_" in name or "_Float16" in name)


def busy(derived_csv: str, raw_csv: str, out_json: str) -> dict:
    """Per-form medians over the dispatches of k_amp_mfma: the derived
    percentages as rocprofv3 computes them and the raw counters."""
    der, raw = _rows(derived_csv), _rows(raw_csv)
    res = {"kernel": "k_amp_mfma",
           "workload": "w20_n1m_k256: 1M events x 20 waves, 256 vectors per pass", "forms": {}}
    for tag, want_bf16 in (("bf16", True), ("fp16", False)):
        form = {}
        for rows in (der, raw):
            names = sorted({r["Kernel_Name"] for r in rows if "k_amp_mfma" in r["Kernel_Name"]
                            and _is_bf16(r["Kernel_Name"]) == want_bf16})
            for r in rows:
                if r["Kernel_Name"] in names:
                    form.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            if names:
                form.setdefault("_names", names)
        res["forms"][tag] = {k: (statistics.median(v) if k != "_names" else v)
                             for k, v in form.items()}
        res["forms"][tag]["dispatches"] = {k: len(v) for k, v in form.items() if k != "_names"}
    with open(out_json, "w") as fo:
        json.dump(res, fo, indent=1)
        fo.write("\n")
    return res


def counters(needle: str, csvs, out_json: str) -> dict:
    """Medians over the dispatches of the kernels named like `needle` of every
    counter in the given rocprofv3 counter-collection files."""
    res = {"kernel": needle, "counters": {}, "dispatches": {}, "names": []}
    vals = {}
    for path in csvs:
        for r in _rows(path):
            if needle in r["Kernel_Name"]:
                vals.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
                if r["Kernel_Name"] not in res["names"]:
                    res["names"].append(r["Kernel_Name"])
    res["counters"] = {k: statistics.median(v) for k, v in vals.items()}
    res["dispatches"] = {k: len(v) for k, v in vals.items()}
    with open(out_json, "w") as fo:
        json.dump(res, fo, indent=1)
        fo.write("\n")
    return res


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "run":
        run(int(sys.argv[2]) if len(sys.argv) > 2 else 5)
    elif len(sys.argv) >= 2 and sys.argv[1] == "run-hess":
        run_hess(int(sys.argv[2]) if len(sys.argv) > 2 else 4)
    elif len(sys.argv) >= 5 and sys.argv[1] == "counters":
        print(json.dumps(counters(sys.argv[2], sys.argv[3:-1], sys.argv[-1]), indent=1))
    elif len(sys.argv) >= 2 and sys.argv[1] == "run-batched":
        run_batched(int(sys.argv[2]) if len(sys.argv) > 2 else 4)
    elif len(sys.argv) == 5 and sys.argv[1] == "busy":
        print(json.dumps(busy(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
    elif len(sys.argv) == 5 and sys.argv[1] == "summarize":
        print(json.dumps(summarize(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
    else:
        raise SystemExit(__doc__)
