"""Summaries of rocprofv3 CSV output (kernel statistics and PMC counters).

    python -m paper_2210_04449_amd.prof_summary stats <dir>/<name>_kernel_stats.csv
    python -m paper_2210_04449_amd.prof_summary pmc <counter_collection.csv> [...]
    python -m paper_2210_04449_amd.prof_summary hash

Only this library's kernels (and the calibration copy) are listed unless
``--all`` is given.

The PMC summary reports counter values per dispatch for each kernel.  HBM
bytes come from FETCH_SIZE and WRITE_SIZE (KiB per dispatch); each is scaled
by what the same counter reads for the device-to-device copy of a known size
that ``bench.py --calibrate-copy`` performs first (256 MiB read, 256 MiB
written; the copy runs as ``__amd_rocclr_copyBuffer``, and it is the largest
dispatch of that kernel in the run).  The summary records the hash of the
tracer's sources it was measured on (``source_hash``: the tracer kernel, the
scene layout it reads and the shared helpers), so a reader can tell whether
the counters still describe the current tracer.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import os
import sys

COPY_BYTES = 256 << 20
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")


# sources that determine the tracer's memory traffic: the kernel, the scene layout it reads, shared helpers
TRACER_SOURCES = ("common.hpp", "scene.hip", "trace.hip")


def source_hash(files=TRACER_SOURCES) -> str:
    """sha256 over the named kernel sources (file names and contents)."""
    h = hashlib.sha256()
    for name in sorted(files):
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_summary(path: str, kernel_prefix: str) -> dict | None:
    """HBM bytes per dispatch of a kernel from a PMC summary, if the summary's source hash is current."""
    try:
        lines = open(path).read().splitlines()
    except OSError:
        return None
    tag = next((ln.split()[-1] for ln in lines if ln.startswith("source_hash")), None)
    if tag != source_hash():
        return None
    for ln in lines:
        if ln.startswith("traffic ") and kernel_prefix in ln.split()[1]:
            f = dict(kv.split("=") for kv in ln.split()[2:])
            return {"fetch_bytes": float(f["fetch_bytes"]), "write_bytes": float(f["write_bytes"])}
    return None


def ours(name: str) -> bool:
    """Kernels of this library, and the device-to-device copy the counters are calibrated with."""
    return "rtsdf::" in name or "copyBuffer" in name


def stats(path: str, keep=ours) -> str:
    rows = [r for r in csv.DictReader(open(path)) if keep(r["Name"])]
    out = [f"{'kernel':<100} {'calls':>5} {'avg_us':>12} {'min_us':>11} {'max_us':>11}"]
    for r in rows:
        out.append(f"{r['Name'][:100]:<100} {r['Calls']:>5} {float(r['AverageNs']) / 1e3:>12.1f} "
                   f"{float(r['MinNs']) / 1e3:>11.1f} {float(r['MaxNs']) / 1e3:>11.1f}")
    return "\n".join(out)


def pmc(paths: list[str], keep=ours) -> str:
    per = collections.defaultdict(lambda: collections.defaultdict(list))  # kernel -> counter -> per dispatch
    for p in paths:
        acc = collections.defaultdict(float)
        names = {}
        for r in csv.DictReader(open(p)):
            if not keep(r["Kernel_Name"]):
                continue
            key = (r["Dispatch_Id"], r["Counter_Name"])
            acc[key] += float(r["Counter_Value"])
            names[r["Dispatch_Id"]] = r["Kernel_Name"]
        for (disp, ctr), v in acc.items():
            per[names[disp]][ctr].append(v)
    out = [f"source_hash {source_hash()}"]
    scale = {}
    for k, cs in per.items():
        if "copyBuffer" in k:
            for c in ("FETCH_SIZE", "WRITE_SIZE"):
                if c in cs:
                    scale[c] = COPY_BYTES / (max(cs[c]) * 1024.0)
    out.append("copy calibration (256 MiB device-to-device): bytes per counted byte = "
               + ", ".join(f"{c} x{v:.3f}" for c, v in sorted(scale.items())))
    for k, cs in sorted(per.items(), key=lambda kv: kv[0]):
        if "FETCH_SIZE" in cs and "WRITE_SIZE" in cs and "FETCH_SIZE" in scale and "WRITE_SIZE" in scale:
            fb = sum(cs["FETCH_SIZE"]) / len(cs["FETCH_SIZE"]) * 1024.0 * scale["FETCH_SIZE"]
            wb = sum(cs["WRITE_SIZE"]) / len(cs["WRITE_SIZE"]) * 1024.0 * scale["WRITE_SIZE"]
            name = k.split("(")[0].replace(" ", "")
            out.append(f"traffic {name} fetch_bytes={fb:.0f} write_bytes={wb:.0f}")
    for k, cs in sorted(per.items(), key=lambda kv: kv[0]):
        out.append(f"\n{k}")
        for c, vals in sorted(cs.items()):
            mean = sum(vals) / len(vals)
            line = f"  {c:<28} per dispatch {mean:>20.1f}  ({len(vals)} dispatches)"
            if c in scale:
                line += f"  -> {mean * 1024.0 * scale[c] / 1e6:.2f} MB"
            out.append(line)
        out.extend(derived(cs))
    return "\n".join(out)


def derived(cs) -> list[str]:
    """Ratios of the counters of one kernel (means per dispatch): L2 hit rate, the share of VALU instruction
    slots' lanes that were active, VALU instructions per wavefront, SALU per VALU instruction."""
    m = {c: sum(v) / len(v) for c, v in cs.items()}
    out = []
    if m.get("TCC_HIT_sum", 0) + m.get("TCC_MISS_sum", 0) > 0:
        out.append(f"  derived L2 hit rate {m['TCC_HIT_sum'] / (m['TCC_HIT_sum'] + m['TCC_MISS_sum']):.3f}")
    if m.get("SQ_ACTIVE_INST_VALU", 0) > 0 and "SQ_THREAD_CYCLES_VALU" in m:
        out.append(f"  derived VALU active-lane fraction {m['SQ_THREAD_CYCLES_VALU'] / (64 * m['SQ_ACTIVE_INST_VALU']):.3f}")
    if m.get("SQ_WAVES", 0) > 0 and "SQ_INSTS_VALU" in m:
        out.append(f"  derived VALU instructions per wavefront {m['SQ_INSTS_VALU'] / m['SQ_WAVES']:.0f}")
    if m.get("SQ_INSTS_VALU", 0) > 0 and "SQ_INSTS_SALU" in m:
        out.append(f"  derived SALU per VALU instruction {m['SQ_INSTS_SALU'] / m['SQ_INSTS_VALU']:.3f}")
    return out


def main(argv):
    if len(argv) == 2 and argv[1] == "hash":
        print(source_hash())
        return 0
    keep = ours
    if "--all" in argv:  # every kernel of the run (torch's too)
        argv = [a for a in argv if a != "--all"]
        keep = lambda name: True  # noqa: E731
    if len(argv) < 3 or argv[1] not in ("stats", "pmc"):
        print(__doc__)
        return 2
    print(stats(argv[2], keep) if argv[1] == "stats" else pmc(argv[2:], keep))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
