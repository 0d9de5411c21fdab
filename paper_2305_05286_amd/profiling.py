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


def lds(a) -> dict:
    """LDS traffic of the CBP kernel from two counter passes.

    a.dir: SQ_INSTS_LDS, SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT,
    SQ_LDS_ADDR_CONFLICT, SQ_ACTIVE_INST_LDS, GRBM_GUI_ACTIVE.  Busy: the
    profiler's own LdsUtil, cycles the LDS serves indexed accesses (summed
    over CUs) over the GPU-active cycles of one XCD times the CUs.
    a.bw: SQ_INSTS_LDS_LOAD_BANDWIDTH and SQ_INSTS_LDS_STORE_BANDWIDTH, the
    bytes the LDS instructions moved (active lanes times access size) in
    units of 64 bytes: the LDS bytes per launch.  The static estimate beside
    it (SQ_INSTS_LDS x 64 lanes x the kernel's mean DS access size, lds_mix)
    cross-checks it."""
    def mean(d, c):
        return statistics.mean(_counter(d, is_cbp, c))
    mix = lds_mix()
    ins = mean(a.dir, "SQ_INSTS_LDS")
    idx, grbm = mean(a.dir, "SQ_LDS_IDX_ACTIVE"), mean(a.dir, "GRBM_GUI_ACTIVE")
    ld, st = mean(a.bw, "SQ_INSTS_LDS_LOAD_BANDWIDTH") * 64, mean(a.bw, "SQ_INSTS_LDS_STORE_BANDWIDTH") * 64
    cus, xcds = 256, 8
    return {"kernel": "qc_reg_kernel<QcGraph0, CBP>", "kernel_hash": kernel_hash(), "ebn0_db": a.ebn0,
            "lds_wave_instructions_per_launch": ins,
            "lds_idx_active_cycles_per_launch": idx,
            "lds_bank_conflict_cycles_per_launch": mean(a.dir, "SQ_LDS_BANK_CONFLICT"),
            "lds_addr_conflict_cycles_per_launch": mean(a.dir, "SQ_LDS_ADDR_CONFLICT"),
            "active_inst_lds_per_launch": mean(a.dir, "SQ_ACTIVE_INST_LDS"),
            "grbm_gui_active_all_xcds": grbm, "lds_busy": idx / cus / (grbm / xcds),
            "lds_load_bytes_per_launch": ld, "lds_store_bytes_per_launch": st,
            "lds_bytes_per_launch": ld + st,
            "lds_bytes_static_estimate": ins * 64 * mix["lds_bytes_per_lane_per_instruction"], **mix}


# bytes per lane moved by each LDS instruction form (gfx9 DS encoding);
# permutes and swizzles go through the LDS crossbar without touching its banks'
# storage and count as one dword
DS_BYTES = {"read_u8": 1, "read_i8": 1, "read_u16": 2, "read_i16": 2, "read_u8_d16": 1,
            "read_u8_d16_hi": 1, "read_u16_d16": 2, "read_u16_d16_hi": 2, "read_b32": 4, "read_b64": 8,
            "read_b96": 12, "read_b128": 16, "read2_b32": 8, "read2st64_b32": 8, "read2_b64": 16,
            "read2st64_b64": 16, "write_b8": 1, "write_b16": 2, "write_b8_d16_hi": 1, "write_b16_d16_hi": 2,
            "write_b32": 4, "write_b64": 8, "write_b96": 12, "write_b128": 16, "write2_b32": 8,
            "write2st64_b32": 8, "write2_b64": 16, "write2st64_b64": 16, "bpermute_b32": 4,
            "permute_b32": 4, "swizzle_b32": 4, "add_u32": 4, "max_u32": 4, "min_u32": 4}


def lds_mix(kernel_symbol_part: str = "qc_reg_kernelINS0_8QcGraph0ELi0ELb0E") -> dict:
    """Static LDS instruction mix of the CBP register-resident kernel: the
    kernel's gfx950 assembly (compiled here with the library's flags) and the
    bytes per lane of each DS instruction in it.  The mean bytes per LDS
    wave-instruction turns the SQ_INSTS_LDS counter into LDS bytes."""
    import re
    import subprocess
    import tempfile
    from paper_2305_05286_amd import build
    flags = [f for f in build.FLAGS if f not in ("-Xarch_device", "-fPIC")]
    with tempfile.TemporaryDirectory() as td:
        out = Path(td) / "k.s"
        subprocess.run([build.HIPCC, *flags, "--cuda-device-only", "-S",
                        str(build.CSRC / "qc_reg.hip"), "-o", str(out)], check=True, capture_output=True)
        text = out.read_text()
    start = text.index(f"_ZN3cbp12_GLOBAL__N_113{kernel_symbol_part}")
    start = text.index("\n", text.index(":", start))
    end = text.index(".Lfunc_end", start)
    counts: dict = {}
    for m in re.finditer(r"\bds_([a-z0-9_]+)", text[start:end]):
        counts[m.group(1)] = counts.get(m.group(1), 0) + 1
    unknown = sorted(k for k in counts if k not in DS_BYTES)
    if unknown:
        raise ValueError(f"unknown DS forms {unknown}")
    n = sum(counts.values())
    byts = sum(DS_BYTES[k] * c for k, c in counts.items())
    return {"ds_static_counts": counts, "ds_static_instructions": n,
            "lds_bytes_per_lane_per_instruction": byts / n}


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
    for name in ("valu", "lds"):
        v = sub.add_parser(name)
        v.add_argument("dir")
        if name == "lds":
            v.add_argument("--bw", required=True, help="pass with the LDS load/store bandwidth counters")
        v.add_argument("--ebn0", type=float, required=True)
        v.add_argument("--out", required=True)
    sub.add_parser("ldsmix")
    an = sub.add_parser("annotate", help="record the counted launch's frame-sweeps in a summary, so that "
                                         "its per-launch counts scale to other launches of the kernel")
    an.add_argument("file")
    an.add_argument("--frame-sweeps", type=float, required=True,
                    help="sweeps summed over the frames of the counted launch")
    a = ap.parse_args()
    if a.cmd == "trace":
        print(trace_table(a.dir))
    elif a.cmd == "ldsmix":
        print(json.dumps(lds_mix(), indent=1))
    elif a.cmd == "annotate":
        f = Path(a.file)
        res = json.loads(f.read_text())
        res["frame_sweeps_per_launch"] = a.frame_sweeps
        f.write_text(json.dumps(res, indent=1) + "\n")
    else:
        res = {"traffic": traffic, "valu": valu, "lds": lds}[a.cmd](a)
        Path(a.out).write_text(json.dumps(res, indent=1) + "\n")
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
