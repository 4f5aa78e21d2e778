"""Summarise rocprofv3 CSV output into short text records.

  python -m paper_2204_03775_amd.profile_summary stats DIR/PREFIX --command CMD --out FILE.md
      kernel-trace statistics (<prefix>_kernel_stats.csv): the kernels by
      total time, with calls and average duration, and, where the kernel
      trace and agent list (<prefix>_kernel_trace.csv, _agent_info.csv) are
      beside it, each kernel's registers, LDS and the occupancy they allow;

  python -m paper_2204_03775_amd.profile_summary kernels --fetch F --write W \\
      --fetch-probe PF --write-probe PW --title T --commands CMDS --out FILE.md
      the same scaling for every library kernel, per kernel and grid size;

  python -m paper_2204_03775_amd.profile_summary counters --csv C --title T --command CMD --out F
      per-kernel averages of any counter set (LDS bank conflicts, issue);

  python -m paper_2204_03775_amd.profile_summary overlap --trace T --match M \
      --window LABEL,FIRST,COUNT [...] --command CMD --out FILE.md
      how much the dispatches of a window (matching kernels in time order,
      FIRST < 0 counting from the end) ran at the same time: hardware
      queues used, busy time over wall time, share of the time with two or
      more running;

  python -m paper_2204_03775_amd.profile_summary traffic \\
      --fetch-step F --write-step W --fetch-probe PF --write-probe PW \\
      --kernel NAME --zchunk ZC --points N --commands CMDS --out-json J --out-md M
      HBM bytes per launch of the step kernel from FETCH_SIZE and WRITE_SIZE
      (KiB per dispatch), each scaled by the factor that maps the same
      counter onto the known traffic of the copy probe (8 bytes per element:
      one read, one write).

The traffic record carries the SHA-256 of the step kernel's sources
(wave_dev.h, wave_step.h, k_fwd_f32.hip) it was taken on; bench.py
reports it only while they are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("wave_dev.h", "wave_step.h", "k_fwd_f32.hip")]


def source_digest() -> str:
    """SHA-256 over the FP32 step kernel's sources (same as bench.py's)."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _short(name: str, n: int = 90) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name if len(name) <= n else name[:n - 3] + "..."


def per_kernel(counter_csv: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    out = collections.defaultdict(list)
    with open(counter_csv) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                out[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return out


# the copy probe's kernel, by its exact name (library kernels such as a
# "direct_copy_kernel" also contain "copy_k")
PROBE_COPY = "::copy_k("


def pick(d, key):
    """The one key of d whose kernel name (the key, or its first element)
    contains key."""
    hits = [k for k in d if key in (k[0] if isinstance(k, tuple) else k)]
    if len(hits) != 1:
        raise SystemExit(f"expected one kernel matching {key!r}, found {hits}")
    return hits[0]


# gfx950 compute unit: 4 SIMDs, at most 8 waves each, 512 vector registers
# per lane in each SIMD (architectural and accumulation registers share them),
# 160 KiB of LDS
SIMDS_PER_CU = 4
MAX_WAVES_PER_SIMD = 8
VGPRS_PER_SIMD_LANE = 512
LDS_BYTES_PER_CU = 160 * 1024


def occupancy(vgpr: int, agpr: int, lds: int, wg_size: int):
    """(work-groups per CU, waves per SIMD) that the vector registers and the
    LDS of one work-group allow.  ``vgpr`` and ``agpr`` are the allocated
    counts per lane (as the kernel trace reports them), ``lds`` the bytes per
    work-group.  Scalar registers are not counted."""
    waves_wg = -(-wg_size // 64)
    regs = vgpr + agpr
    per_simd = MAX_WAVES_PER_SIMD if regs == 0 else min(MAX_WAVES_PER_SIMD, VGPRS_PER_SIMD_LANE // regs)
    slots = SIMDS_PER_CU * per_simd  # waves a CU holds at this register count
    wgs = slots // waves_wg
    if lds > 0:
        wgs = min(wgs, LDS_BYTES_PER_CU // lds)
    return wgs, wgs * waves_wg / SIMDS_PER_CU


# GPUs whose kernels allocate vector registers in granules of 8 (one
# 512-register file per SIMD lane).  The kernel trace prints the count
# decoded with a granule of 4, half the allocation: the compiler's resource
# report for the same kernels gives 130, 176 and 186 registers where the
# trace prints 68, 88 and 96 (each rounded up to 8, then halved).
GRANULE8_TARGETS = ("gfx90a", "gfx942", "gfx950")


def allocated_vgprs(printed: int, target: str) -> int:
    return 2 * printed if target in GRANULE8_TARGETS else printed


def resources(trace_csv: str, names, target: str = ""):
    """Resource rows (registers, LDS, work-group size, occupancy) of the
    kernels ``names``, from a kernel trace (the first dispatch of each) of a
    GPU of ISA ``target``."""
    first = {}
    with open(trace_csv) as f:
        for r in csv.DictReader(f):
            if r["Kernel_Name"] in names and r["Kernel_Name"] not in first:
                first[r["Kernel_Name"]] = r
    lines = ["", f"Resources on {target or 'the GPU'} (first dispatch of each kernel).  Vector registers as "
             "allocated per lane",
             "(twice the count the trace prints on this GPU, which decodes it with a granule of 4 instead of 8);",
             "occupancy from the registers and LDS alone: 4 SIMDs per CU, at most 8 waves and 512 registers",
             "per lane each, 160 KiB of LDS:", "",
             "| kernel | VGPR | AGPR | SGPR | LDS bytes | scratch | work-group | work-groups launched | "
             "work-groups / CU | waves / SIMD |",
             "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for n in names:
        r = first.get(n)
        if r is None:
            continue
        v = allocated_vgprs(int(r["VGPR_Count"]), target)
        # accumulation registers as printed (none of the library's kernels uses any)
        acc = int(r["Accum_VGPR_Count"])
        lds = int(r["LDS_Block_Size"])
        wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        wgs, waves = occupancy(v, acc, lds, wg)
        lines.append(f"| `{_short(n)}` | {v} | {acc} | {r['SGPR_Count']} | {lds} | {r['Scratch_Size']} | {wg} | "
                     f"{-(-grid // wg)} | {wgs} | {waves:g} |")
    return lines


def gpu_target(agent_csv: str) -> str:
    """ISA name of the first GPU agent in an agent-info file."""
    with open(agent_csv) as f:
        for r in csv.DictReader(f):
            if r["Name"].startswith("gfx"):
                return r["Name"]
    return ""


def stats(prefix: str, command: str, out: str):
    rows = list(csv.DictReader(open(prefix + "_kernel_stats.csv")))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
             "| kernel | calls | total ms | average us | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows[:12]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    if os.path.exists(prefix + "_kernel_trace.csv") and os.path.exists(prefix + "_agent_info.csv"):
        lines += resources(prefix + "_kernel_trace.csv", [r["Name"] for r in rows[:12]],
                           gpu_target(prefix + "_agent_info.csv"))
    open(out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def overlap_of(rows):
    """(dispatches, hardware queues, summed durations, wall span, time with
    two or more dispatches running), times in ns, of kernel-trace rows."""
    ev = []
    for r in rows:
        ev.append((int(r["Start_Timestamp"]), 1))
        ev.append((int(r["End_Timestamp"]), -1))
    ev.sort()  # at equal times an end (-1) comes before a start
    active, last, multi = 0, None, 0
    for t, d in ev:
        if last is not None and active >= 2:
            multi += t - last
        active += d
        last = t
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in rows)
    span = (ev[-1][0] - ev[0][0]) if ev else 0
    return len(rows), len({r["Queue_Id"] for r in rows}), busy, span, multi


def overlap(a):
    rows = [r for r in csv.DictReader(open(a.trace)) if a.match in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    lines = ["# Concurrency of kernel dispatches (rocprofv3 kernel trace)", "",
             f"Command: `{a.command}`", "",
             f"Dispatches of kernels matching `{a.match}`, in start order; a window is "
             "(first, count), first < 0 counting from the end.", "",
             "| window | first, count | dispatches | hardware queues | busy ms | wall ms | busy / wall | "
             "share of wall with >= 2 running |",
             "|---|---|---:|---:|---:|---:|---:|---:|"]
    for spec in a.window:
        label, first, count = spec.rsplit(",", 2)
        first, count = int(first), int(count)
        start = first if first >= 0 else len(rows) + first
        w = rows[start:start + count]
        n, q, busy, span, multi = overlap_of(w)
        lines.append(f"| {label} | {first}, {count} | {n} | {q} | {busy / 1e6:.1f} | {span / 1e6:.1f} | "
                     f"{busy / max(span, 1):.2f} | {multi / max(span, 1):.2f} |")
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def traffic(a):
    fs = per_kernel(a.fetch_step, "FETCH_SIZE")
    ws = per_kernel(a.write_step, "WRITE_SIZE")
    fp = per_kernel(a.fetch_probe, "FETCH_SIZE")
    wp = per_kernel(a.write_probe, "WRITE_SIZE")
    ks, kp = pick(fs, a.match), pick(fp, PROBE_COPY)
    avg = lambda v: sum(v) / len(v)
    copy_kib = a.probe_elements * 4 / 1024.0  # bytes read (= bytes written) by one copy
    f_scale = copy_kib / avg(fp[kp])
    w_scale = copy_kib / avg(wp[pick(wp, PROBE_COPY)])
    fetch_b = avg(fs[ks]) * f_scale * 1024
    write_b = avg(ws[pick(ws, a.match)]) * w_scale * 1024
    algo_read, algo_write = 12 * a.points, 4 * a.points
    rec = {
        "kernel": a.kernel, "zchunk": a.zchunk,
        "source_sha256": source_digest(),
        "dispatches": len(fs[ks]),
        "fetch_kib_per_dispatch": round(avg(fs[ks]), 1),
        "write_kib_per_dispatch": round(avg(ws[pick(ws, a.match)]), 1),
        "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4),
        "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
        "bytes_per_launch": round(fetch_b + write_b),
        "algorithmic_bytes_per_launch": algo_read + algo_write,
        "read_excess": round(fetch_b / algo_read, 4), "write_excess": round(write_b / algo_write, 4),
        "commands": a.commands,
    }
    json.dump(rec, open(a.out_json, "w"), indent=1)
    lines = [
        "# HBM traffic of the step kernel (rocprofv3 counters)", "",
        f"Kernel `{_short(ks)}` = variant `{a.kernel}`, z-chunk {a.zchunk}, "
        f"{a.points} interior updates per launch, {rec['dispatches']} dispatches.", "",
        "Scale factors come from the copy probe (`copy_k`, "
        f"{a.probe_elements} floats: {copy_kib:.0f} KiB read and written): "
        f"FETCH_SIZE x {f_scale:.4f}, WRITE_SIZE x {w_scale:.4f}.", "",
        "| quantity | per launch |", "|---|---:|",
        f"| FETCH_SIZE (KiB, raw) | {rec['fetch_kib_per_dispatch']} |",
        f"| WRITE_SIZE (KiB, raw) | {rec['write_kib_per_dispatch']} |",
        f"| bytes read (scaled) | {fetch_b / 1e9:.4f} GB = {rec['read_excess']:.3f} x algorithmic 12 B/pt |",
        f"| bytes written (scaled) | {write_b / 1e9:.4f} GB = {rec['write_excess']:.3f} x algorithmic 4 B/pt |",
        f"| total | {(fetch_b + write_b) / 1e9:.4f} GB vs algorithmic {(algo_read + algo_write) / 1e9:.4f} GB |",
        "", "Commands:", ""] + [f"    {c}" for c in a.commands]
    open(a.out_md, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def kernels(a):
    """Scaled read / write bytes per dispatch of every library kernel, per
    launch size (kernels of one name and grid size are averaged together)."""
    def per(path, ctr):
        d = collections.defaultdict(list)
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == ctr:
                    d[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
        return d
    fs, ws = per(a.fetch, "FETCH_SIZE"), per(a.write, "WRITE_SIZE")
    fp, wp = per(a.fetch_probe, "FETCH_SIZE"), per(a.write_probe, "WRITE_SIZE")
    avg = lambda v: sum(v) / len(v)
    copy_kib = a.probe_elements * 4 / 1024.0
    f_scale = copy_kib / avg(fp[pick(fp, PROBE_COPY)])
    w_scale = copy_kib / avg(wp[pick(wp, PROBE_COPY)])
    lines = [f"# {a.title}", "",
             f"FETCH_SIZE x {f_scale:.4f} and WRITE_SIZE x {w_scale:.4f} (copy probe, "
             f"{a.probe_elements} floats).  Rows group dispatches by kernel and grid size.", "",
             "| kernel | grid (work-items) | dispatches | read MB / dispatch | written MB / dispatch |",
             "|---|---:|---:|---:|---:|"]
    rows = sorted(((k, v) for k, v in fs.items() if a.match in k[0]), key=lambda kv: -avg(kv[1]) * len(kv[1]))
    for (name, grid), v in rows:
        w = ws.get((name, grid), [0.0])
        lines.append(f"| `{_short(name, 70)}` | {grid} | {len(v)} | {avg(v) * f_scale * 1024 / 1e6:.2f} | "
                     f"{avg(w) * w_scale * 1024 / 1e6:.2f} |")
    lines += ["", "Commands:", ""] + [f"    {c}" for c in a.commands]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def counters(a):
    """Average of every counter per dispatch, per kernel and grid size, for
    the library's kernels; with the LDS counters present, the bank-conflict
    ratio SQ_LDS_BANK_CONFLICT / (SQ_LDS_IDX_ACTIVE - SQ_LDS_BANK_CONFLICT)
    (conflict cycles per conflict-free LDS cycle)."""
    d = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(a.csv) as f:
        for r in csv.DictReader(f):
            if a.match in r["Kernel_Name"]:
                d[(r["Kernel_Name"], int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for v in d.values() for c in v})
    lines = [f"# {a.title}", "", "Averages per dispatch (counters summed over the GPU).", "",
             "| kernel | grid | dispatches | " + " | ".join(names) + (" | LDS conflict ratio |" if "SQ_LDS_BANK_CONFLICT" in names else " |"),
             "|---|---:|---:|" + "---:|" * len(names) + ("---:|" if "SQ_LDS_BANK_CONFLICT" in names else "")]
    for (name, grid), v in sorted(d.items(), key=lambda kv: kv[0]):
        av = {c: sum(x) / len(x) for c, x in v.items()}
        n = max(len(x) for x in v.values())
        row = f"| `{_short(name, 60)}` | {grid} | {n} | " + " | ".join(f"{av.get(c, 0):.4g}" for c in names)
        if "SQ_LDS_BANK_CONFLICT" in names:
            act, bc = av.get("SQ_LDS_IDX_ACTIVE", 0.0), av.get("SQ_LDS_BANK_CONFLICT", 0.0)
            row += f" | {bc / (act - bc):.4f}" if act > bc else " | -"
        lines.append(row + " |")
    lines += ["", "Command:", "", f"    {a.command}"]
    open(a.out, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("prefix")
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch-step", "write-step", "fetch-probe", "write-probe", "kernel", "out-json", "out-md"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--zchunk", type=int, required=True)
    t.add_argument("--match", default="step_tiled<0, 64, 8, 1>",
                   help="kernel name substring (the FP32 step kernel of the variant)")
    t.add_argument("--points", type=int, required=True)
    t.add_argument("--probe-elements", type=int, required=True)
    t.add_argument("--commands", nargs="+", required=True)
    k = sub.add_parser("kernels")
    for name in ("fetch", "write", "fetch-probe", "write-probe", "out", "title"):
        k.add_argument("--" + name, required=True)
    k.add_argument("--match", default="wavek::")
    k.add_argument("--probe-elements", type=int, required=True)
    k.add_argument("--commands", nargs="+", required=True)
    c = sub.add_parser("counters")
    for name in ("csv", "out", "title", "command"):
        c.add_argument("--" + name, required=True)
    c.add_argument("--match", default="wavek::")
    o = sub.add_parser("overlap")
    for name in ("trace", "match", "command", "out"):
        o.add_argument("--" + name, required=True)
    o.add_argument("--window", action="append", required=True, help="LABEL,FIRST,COUNT")
    a = ap.parse_args()
    if a.cmd == "overlap":
        overlap(a)
    elif a.cmd == "counters":
        counters(a)
    elif a.cmd == "stats":
        stats(a.prefix, a.command, a.out)
    elif a.cmd == "kernels":
        kernels(a)
    else:
        traffic(a)


if __name__ == "__main__":
    main()
