"""Summaries of rocprofv3 output for the committed profiles.

  python -m paper_2305_05286_amd.profiling trace DIR            # --kernel-trace --stats -f csv
  python -m paper_2305_05286_amd.profiling traffic --fetch D1 --write D2 \\
      --copy-fetch D3 --copy-write D4 --ebn0 1.75 --out profiles/traffic_qc2304_cbp.json
  python -m paper_2305_05286_amd.profiling valu D --ebn0 1.75 --out profiles/valu_qc2304_cbp.json

`traffic` reads FETCH_SIZE and WRITE_SIZE (KiB per dispatch, one counter pass
each) of the CBP register-resident kernel and scales each by what the same
counter reads for a plain device copy of known size (1 GiB read + 1 GiB
written, `bench.py --copy-calibration`), giving HBM bytes per launch.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import statistics
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]
KERNEL_SOURCES = ["paper_2305_05286_amd/csrc/qc_reg.hip", "paper_2305_05286_amd/csrc/phi.hpp"]
COPY_BYTES = 1 << 30


def kernel_hash() -> str:
    """Hash of the CBP kernel's sources and compile flags (counter files carry it)."""
    from paper_2305_05286_amd import build
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update((ROOT / p).read_bytes())
    h.update(" ".join(f for f in build.FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    n = name.replace("cbp::(anonymous namespace)::", "")
    n = n.replace("(anonymous namespace)::", "")
    if "QcArgs" in n:
        n = n.split("(")[0].replace("void ", "")
    if "StreamArgs" in n or "SparseDev" in n:
        n = n.split("(")[0].replace("void ", "")
    return n[:90]


def _csv(pattern: str):
    files = glob.glob(pattern, recursive=True)
    if not files:
        raise FileNotFoundError(pattern)
    with open(files[0]) as fh:
        return list(csv.DictReader(fh))


def trace_table(d: str) -> str:
    rows = _csv(f"{d}/**/*kernel_stats.csv")
    out = ["| kernel | calls | avg ms | min ms | max ms | % time |", "|---|---|---|---|---|---|"]
    for r in rows[:12]:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['MinNs']) / 1e6:.3f} | {float(r['MaxNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out)


def _counter(d: str, match, counter: str):
    vals = [float(r["Counter_Value"]) for r in _csv(f"{d}/**/*counter_collection.csv")
            if match(r["Kernel_Name"]) and r["Counter_Name"] == counter]
    if not vals:
        raise ValueError(f"no {counter} rows in {d}")
    return vals


def is_cbp(n: str) -> bool:
    return "qc_reg_kernel" in n and "QcGraph0, 0, false" in n


def is_stream_cbp(n: str) -> bool:
    return "qc_stream_kernel<0, false>" in n or ("qc_stream_kernel" in n and "ILi0ELb0E" in n)


MATCHERS = {"qc_reg": (is_cbp, "qc_reg_kernel<QcGraph0, CBP>"),
            "qc_stream": (is_stream_cbp, "qc_stream_kernel<CBP> (n=26112)")}


def is_copy(n: str) -> bool:
    # torch's contiguous device-to-device copy runs the runtime's blit kernel
    return n.startswith("__amd_rocclr_copyBuffer")


def traffic(a) -> dict:
    match, label = MATCHERS[a.kernel]
    fetch = _counter(a.fetch, match, "FETCH_SIZE")
    write = _counter(a.write, match, "WRITE_SIZE")
    cf = max(_counter(a.copy_fetch, is_copy, "FETCH_SIZE"))
    cw = max(_counter(a.copy_write, is_copy, "WRITE_SIZE"))
    kf = COPY_BYTES / (cf * 1024.0)
    kw = COPY_BYTES / (cw * 1024.0)
    fb = statistics.mean(fetch) * 1024.0 * kf
    wb = statistics.mean(write) * 1024.0 * kw
    return {"kernel": label, "kernel_hash": kernel_hash() if a.kernel == "qc_reg" else None,
            "ebn0_db": a.ebn0, "fetch_kib_per_dispatch": statistics.mean(fetch),
            "write_kib_per_dispatch": statistics.mean(write),
            "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_scale": kf, "write_scale": kw,
            "hbm_read_bytes_per_launch": fb, "hbm_write_bytes_per_launch": wb,
            "hbm_bytes_per_launch": fb + wb}


def valu(a) -> dict:
    """VALU / LDS instruction counts of the CBP kernel (one counter pass).

    gfx950 executes transcendentals (v_exp_f32, v_log_f32) in their own unit,
    overlapped with the main VALU pipeline, so the issue bound of the main
    pipe counts SQ_INSTS_VALU - SQ_INSTS_VALU_TRANS_F32.  VALU busy follows
    the profiler's own derived metric: SQ_ACTIVE_INST_VALU (quad-cycles, summed
    over all SIMDs) per CU over the GPU-active cycles of one XCD.
    """
    def mean(c):
        return statistics.mean(_counter(a.dir, is_cbp, c))
    ins, trans = mean("SQ_INSTS_VALU"), mean("SQ_INSTS_VALU_TRANS_F32")
    active, grbm = mean("SQ_ACTIVE_INST_VALU"), mean("GRBM_GUI_ACTIVE")
    cus, xcds = 256, 8
    return {"kernel": "qc_reg_kernel<QcGraph0, CBP>", "kernel_hash": kernel_hash(),
            "ebn0_db": a.ebn0, "valu_wave_instructions_per_launch": ins,
            "trans_wave_instructions_per_launch": trans,
            "main_valu_wave_instructions_per_launch": ins - trans,
            "lds_wave_instructions_per_launch": mean("SQ_INSTS_LDS"),
            "waves_per_launch": mean("SQ_WAVES"),
            "active_inst_valu_quad_cycles": active, "grbm_gui_active_all_xcds": grbm,
            "valu_busy": active / cus / (grbm / xcds)}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    c = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        c.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    c.add_argument("--ebn0", type=float, required=True)
    c.add_argument("--kernel", choices=sorted(MATCHERS), default="qc_reg")
    c.add_argument("--out", required=True)
    v = sub.add_parser("valu")
    v.add_argument("dir")
    v.add_argument("--ebn0", type=float, required=True)
    v.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace_table(a.dir))
    else:
        res = traffic(a) if a.cmd == "traffic" else valu(a)
        Path(a.out).write_text(json.dumps(res, indent=1) + "\n")
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
