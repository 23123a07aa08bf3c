"""Summarise rocprofv3 runs of bench.py into the committed profile record.

    python -m paper_2110_13055_amd.profile_summary \\
        --trace DIR --fetch DIR --write DIR --bench-log FILE --copy-mib 1024 \\
        --md OUT.md --json OUT.json [--command TEXT ...]

Inputs are the CSV directories of rocprofv3 runs of the same bench command
(``--kernel-trace --stats``, ``--pmc FETCH_SIZE``, ``--pmc WRITE_SIZE`` and,
optionally, ``--pmc TCC_EA0_RDREQ_32B TCC_EA0_RDREQ_64B TCC_EA0_RDREQ_128B``,
all with ``--output-format csv``) and the bench's own stdout
(for the fluid-node count). The bench command must include
``--copy-probe-mib N``: one pass of the bandwidth probe's streaming copy
kernel over N MiB, whose counter readings give the scale from each counter
to bytes (the copy reads and writes exactly N MiB, in 16-byte accesses).

Output: a Markdown table per step-kernel variant (average duration, HBM
bytes per launch and per fluid node from the counters, achieved GB/s) and a
JSON record that bench.py reads for ``roofline.traffic`` (ignored once the
kernel sources change: the record carries their hash).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("step.hip", "device_common.h", "cdi_internal.h")
STORAGE = {"0": "fp32", "1": "fp16_dev", "2": "moments", "3": "fp16"}


def kernel_source_hash() -> str:
    """Hash of the step kernel's sources (a profile is valid for these only)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _variant(name: str):
    """step_kernel<L, ST, ODD, LBM, NP, STG> -> readable label, or None."""
    m = re.search(r"step_kernel<cdi::(D2Q9|D3Q19), (\d), (\d), (\d), (\d)(?:, (\d))?>", name)
    if not m:
        return None
    lat, st, odd, lbm, np_, stg = m.groups()
    kind = "fused" if lbm == "1" and np_ == "1" else ("lbm" if lbm == "1" else "np")
    # ion-only steps and moment storage have no AA parity; 2 = pull streaming
    if kind == "np" or st == "2":
        parity = ""
    else:
        parity = {"0": " even", "1": " odd", "2": " pull"}[odd]
    return f"{lat} {STORAGE[st]} {kind}{parity}{' staged' if stg == '1' else ''}"


def _csv(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def _find(d, suffix):
    for root, _, files in os.walk(d):
        for f in files:
            if f.endswith(suffix):
                return os.path.join(root, f)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def _counters(d, counter):
    """Per-variant mean counter value per dispatch, and the copy probe's value."""
    per = defaultdict(list)
    copy = None
    for r in _csv(_find(d, "counter_collection.csv")):
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        if "copy_kernel(" in r["Kernel_Name"]:
            if copy is None or v > copy:
                copy = v  # the bandwidth probe's streaming copy (the largest of the run)
            continue
        k = _variant(r["Kernel_Name"])
        if k:
            per[k].append(v)
    return {k: sum(v) / len(v) for k, v in per.items()}, copy


RDREQ = {"TCC_EA0_RDREQ_32B": 32.0, "TCC_EA0_RDREQ_64B": 64.0, "TCC_EA0_RDREQ_128B": 128.0}


def _read_requests(d):
    """Per-variant mean HBM read bytes per dispatch from the L2's memory read
    requests by size (32, 64 and 128 bytes; exact for the probe's copy, where
    FETCH_SIZE counts each 128-byte request as 64 bytes)."""
    per = defaultdict(lambda: defaultdict(list))
    for r in _csv(_find(d, "counter_collection.csv")):
        size = RDREQ.get(r["Counter_Name"])
        k = _variant(r["Kernel_Name"])
        if size is None or not k:
            continue
        per[k][r["Counter_Name"]].append(float(r["Counter_Value"]) * size)
    return {k: sum(sum(v) / len(v) for v in byname.values()) for k, byname in per.items()}


def summarise(trace, fetch, write, bench_log, copy_mib, commands=(), rdreq=None):
    stats = {}
    for r in _csv(_find(trace, "kernel_stats.csv")):
        k = _variant(r["Name"])
        if k:
            stats[k] = (int(r["Calls"]), float(r["AverageNs"]) * 1e-9)
    n_fluid = None
    with open(bench_log) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{") and '"n_fluid"' in line:
                n_fluid = json.loads(line)["config"]["n_fluid"]
    if n_fluid is None:
        raise ValueError("bench log holds no result line with config.n_fluid")
    fr, fcopy = _counters(fetch, "FETCH_SIZE")
    wr, wcopy = _counters(write, "WRITE_SIZE")
    copy_bytes = copy_mib * 1024.0 * 1024.0
    fscale = copy_bytes / fcopy  # bytes per counter unit
    wscale = copy_bytes / wcopy
    rq = _read_requests(rdreq) if rdreq else {}
    rows = []
    for k in sorted(stats):
        calls, dur = stats[k]
        fetch_b = fr.get(k, float("nan")) * fscale
        fb = rq.get(k, fetch_b)  # the request counts where taken: exact at every request size
        wb = wr.get(k, float("nan")) * wscale
        rows.append(dict(kernel=k, calls=calls, avg_ms=dur * 1e3, read_bytes=fb, write_bytes=wb,
                         read_per_node=fb / n_fluid, write_per_node=wb / n_fluid,
                         fetch_scaled_per_node=fetch_b / n_fluid, gbs=(fb + wb) / dur / 1e9))
    # bytes per launch of a whole step (the mean of the kernels one step can
    # be: AA even and odd alternate; pull and moment storage use one)
    per_launch = {}
    for st in STORAGE.values():
        for kind in ("fused", "lbm"):
            pair = [r for r in rows if r["kernel"].split()[1:3] == [st, kind]]
            if pair:
                per_launch.setdefault(st, {})[kind] = sum(r["read_bytes"] + r["write_bytes"]
                                                         for r in pair) / len(pair)
    record = dict(kernel_source_hash=kernel_source_hash(), n_fluid=n_fluid,
                  counter_scale={"FETCH_SIZE": fscale, "WRITE_SIZE": wscale},
                  bytes_per_launch={st: v.get("fused") for st, v in per_launch.items()},
                  lbm_bytes_per_launch={st: v.get("lbm") for st, v in per_launch.items()},
                  kernels=rows, commands=list(commands))
    md = [f"# Step kernels on the 512^3 electrode ({n_fluid} fluid nodes)", "",
          f"Kernel source hash: `{record['kernel_source_hash']}`.", "",
          "Counter scale from the bandwidth probe's streaming copy kernel (one pass over "
          f"{copy_mib} MiB, which reads and writes exactly that much): FETCH_SIZE x {fscale:.1f} B, "
          f"WRITE_SIZE x {wscale:.1f} B per unit.", "",
          ("HBM read bytes: the L2's memory read requests by size (32, 64, 128 B), which are exact for the "
           "copy; the FETCH_SIZE column is that counter times the copy's scale, which overstates reads made "
           "of 32- or 64-byte requests." if rq else "HBM read bytes: FETCH_SIZE times the copy's scale."), "",
          "| kernel | calls | avg ms | HBM read B/node | (FETCH_SIZE scaled) | HBM write B/node | achieved GB/s |",
          "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        md.append(f"| {r['kernel']} | {r['calls']} | {r['avg_ms']:.3f} | {r['read_per_node']:.1f} | "
                  f"{r['fetch_scaled_per_node']:.1f} | {r['write_per_node']:.1f} | {r['gbs']:.0f} |")
    md += ["", "Commands (repository root; runs of the same bench command):", ""]
    md += [f"    {c}" for c in commands]
    return record, "\n".join(md) + "\n"


STALL_COUNTERS = ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_LDS")


def summarise_stalls(dirs, commands=()):
    """Per step-kernel variant, from SQ counter passes (each directory one
    rocprofv3 --pmc run, each holding SQ_WAVES): instructions issued per wave
    (VALU, SALU, vector-memory reads and writes, LDS), the fraction of wave
    cycles spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES). A wave covers 64
    fluid nodes. Totals over all dispatches of a
    variant, divided by that pass's total of SQ_WAVES."""
    tot = defaultdict(lambda: defaultdict(float))
    waves = defaultdict(lambda: defaultdict(float))
    for d in dirs:
        for r in _csv(_find(d, "counter_collection.csv")):
            k = _variant(r["Kernel_Name"])
            if not k:
                continue
            v = float(r["Counter_Value"])
            if r["Counter_Name"] == "SQ_WAVES":
                waves[k][d] += v
            else:
                tot[k][(r["Counter_Name"], d)] += v
    rows = []
    for k in sorted(tot):
        row = {"variant": k}
        for (cn, d), v in tot[k].items():
            w = waves[k].get(d)
            if w:
                row[cn] = v / w
        if "SQ_WAIT_ANY" in row and "SQ_WAVE_CYCLES" in row:
            row["wait_fraction"] = row["SQ_WAIT_ANY"] / row["SQ_WAVE_CYCLES"]
        rows.append(row)
    md = ["# Step kernels on the 512^3 electrode: instructions per wave and waiting", "",
          "Per wave (64 fluid nodes), from the SQ counters; waiting = SQ_WAIT_ANY / SQ_WAVE_CYCLES.", "",
          "| kernel | VALU | SALU | VMEM read | VMEM write | LDS | waiting |",
          "|---|---:|---:|---:|---:|---:|---:|"]
    for r in rows:
        def f(c):
            return f"{r[c]:.0f}" if c in r else "-"
        wf = f"{100 * r['wait_fraction']:.0f} %" if "wait_fraction" in r else "-"
        md.append(f"| {r['variant']} | {f('SQ_INSTS_VALU')} | {f('SQ_INSTS_SALU')} | "
                  f"{f('SQ_INSTS_VMEM_RD')} | {f('SQ_INSTS_VMEM_WR')} | {f('SQ_INSTS_LDS')} | {wf} |")
    md += ["", "Commands (repository root):", ""] + [f"    {c}" for c in commands]
    return {"kernels": rows, "commands": list(commands)}, "\n".join(md) + "\n"


def main_stalls(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("--stalls", action="store_true")
    ap.add_argument("--pmc", action="append", required=True, help="a rocprofv3 --pmc output directory")
    ap.add_argument("--md", required=True)
    ap.add_argument("--json", required=True)
    ap.add_argument("--command", action="append", default=[])
    a = ap.parse_args(argv)
    rec, md = summarise_stalls(a.pmc, a.command)
    with open(a.json, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    with open(a.md, "w") as fh:
        fh.write(md)


def main():
    if "--stalls" in sys.argv[1:]:
        return main_stalls(sys.argv[1:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--bench-log", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--md", required=True)
    ap.add_argument("--json", required=True)
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--rdreq", default=None,
                    help="a rocprofv3 --pmc TCC_EA0_RDREQ_32B TCC_EA0_RDREQ_64B TCC_EA0_RDREQ_128B run "
                         "of the same command (exact read bytes)")
    ap.add_argument("--potential", action="store_true",
                    help="summarise the potential-solve kernels (bench.py --potential-only)")
    a = ap.parse_args()
    if a.potential:
        rec, md = summarise_potential(a.trace, a.fetch, a.write, a.bench_log, a.copy_mib, a.command, a.rdreq)
    else:
        rec, md = summarise(a.trace, a.fetch, a.write, a.bench_log, a.copy_mib, a.command, a.rdreq)
    with open(a.json, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    with open(a.md, "w") as fh:
        fh.write(md)



# ---------------------------------------------------------------- potential solve

# per-iteration kernels of the two iterative solvers: role and algorithmic
# bytes per fluid node (the bench's byte model)
POT_KERNELS = {"pot_dirspmv_kernel": ("direction + A p (stencil), FP32 vectors", 41),
               "pot_axpy_kernel": ("x, r update, FP32 vectors", 25)}
# the same CG on FP64 vectors (cdi_potential.fp64 = 1, or a round handed over)
POT64_KERNELS = {"pot_dirspmv_kernel<double>": ("direction + A p (stencil), FP64 vectors", 57),
                 "pot_axpy_kernel<double>": ("x, r update, FP64 vectors", 49)}
# once per refinement round of the potential solve (not per iteration)
POT_ROUND_KERNELS = {"pot_refine_kernel": ("FP64 residual b - A x, FP32 correction start", 53),
                     "pot_correct_kernel": ("x += FP32 correction", 20)}
NPS_KERNELS = {"nps_dir_kernel": ("direction p^ = K^-1 p", 72),
               "nps_apply_kernel<0>": ("v = A p^", 78),
               "nps_sdir_kernel": ("s^ = K^-1 (r - alpha v)", 56),
               "nps_apply_kernel<1>": ("t = A s^", 70),
               "nps_update_kernel": ("x, r update", 120)}


def _solver_kernel(name: str):
    m = re.search(r"nps_apply_kernel<[^,>]+, (\d)>", name)
    if m:
        return f"nps_apply_kernel<{m.group(1)}>"
    m = re.search(r"(pot_dirspmv_kernel|pot_axpy_kernel)<(?:[^<>]*, )?double>", name)
    if m:
        return f"{m.group(1)}<double>"
    for k in list(POT_KERNELS) + list(POT_ROUND_KERNELS) + list(NPS_KERNELS):
        if "<" not in k and k in name:
            return k
    return None


def summarise_potential(trace, fetch, write, bench_log, copy_mib, commands=(), rdreq=None):
    """Per-iteration kernels of the potential solve (Jacobi-PCG) and of the
    implicit ion solve (BiCGSTAB): mean duration, HBM bytes per fluid node and
    GB/s over the dispatches that did work (launches after the device-side
    stop return at once and are left out: below 5% of the kernel's longest
    dispatch)."""
    durs = defaultdict(list)
    for r in _csv(_find(trace, "kernel_trace.csv")):
        k = _solver_kernel(r["Kernel_Name"])
        if k:
            durs[k].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9)
    n_fluid = None
    with open(bench_log) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith("{") and '"potential"' in line:
                n_fluid = json.loads(line)["potential"]["n_fluid"]
    if n_fluid is None:
        raise ValueError("bench log holds no potential record with n_fluid")

    def counters(d, counter):
        per, copy = defaultdict(list), None
        for r in _csv(_find(d, "counter_collection.csv")):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if "copy_kernel(" in r["Kernel_Name"]:
                copy = v if copy is None or v > copy else copy
                continue
            k = _solver_kernel(r["Kernel_Name"])
            if k:
                per[k].append(v)
        out = {}
        for k, v in per.items():
            top = max(v)
            work = [x for x in v if x >= 0.05 * top]
            out[k] = sum(work) / len(work)
        return out, copy

    def read_requests(d):
        per = defaultdict(float)
        for r in _csv(_find(d, "counter_collection.csv")):
            size = RDREQ.get(r["Counter_Name"])
            k = _solver_kernel(r["Kernel_Name"])
            if size is not None and k:
                per[(k, r["Dispatch_Id"])] += float(r["Counter_Value"]) * size
        byk = defaultdict(list)
        for (k, _), v in per.items():
            byk[k].append(v)
        out = {}
        for k, v in byk.items():
            top = max(v)
            work = [x for x in v if x >= 0.05 * top]
            out[k] = sum(work) / len(work)
        return out

    fr, fcopy = counters(fetch, "FETCH_SIZE")
    wr, wcopy = counters(write, "WRITE_SIZE")
    copy_bytes = copy_mib * 1024.0 * 1024.0
    fscale, wscale = copy_bytes / fcopy, copy_bytes / wcopy
    rq = read_requests(rdreq) if rdreq else {}

    def group(kernels):
        rows = []
        for k, (role, alg) in kernels.items():
            if k not in durs:
                continue
            top = max(durs[k])
            work = [x for x in durs[k] if x >= 0.05 * top]
            dur = sum(work) / len(work)
            fb, wb = rq.get(k, fr.get(k, float("nan")) * fscale), wr.get(k, float("nan")) * wscale
            rows.append(dict(kernel=k, role=role, dispatches=len(work), avg_ms=dur * 1e3, alg_per_node=alg,
                             read_per_node=fb / n_fluid, write_per_node=wb / n_fluid, gbs=(fb + wb) / dur / 1e9,
                             alg_gbs=alg * n_fluid / dur / 1e9))
        return rows

    record = dict(n_fluid=n_fluid, counter_scale={"FETCH_SIZE": fscale, "WRITE_SIZE": wscale},
                  commands=list(commands))
    md = [f"# Iterative solvers on the 512^3 electrode ({n_fluid} fluid nodes)", "",
          "Counter scale from the bandwidth probe's streaming copy kernel: FETCH_SIZE x "
          f"{fscale:.1f} B, WRITE_SIZE x {wscale:.1f} B per unit. Algorithmic bytes: what each kernel must move "
          "per fluid node; measured: the HBM counters"
          + (" (reads: the L2's memory read requests by size, exact at every size)." if rq else
             " (reads: FETCH_SIZE times the copy's scale)."), ""]
    for key, title, kernels in (("cg", "Potential, Eq. 4-5: Jacobi-PCG iterations of the mixed-precision refinement",
                                 POT_KERNELS),
                                ("cg64", "Potential: the same CG on FP64 vectors alone (fp64 = 1)", POT64_KERNELS),
                                ("bicgstab", "Steady ion state (implicit scheme): BiCGSTAB, both species, FP64",
                                 NPS_KERNELS)):
        rows = group(kernels)
        if not rows:
            continue
        it_ms = sum(r["avg_ms"] for r in rows)
        it_bytes = sum(r["read_per_node"] + r["write_per_node"] for r in rows)
        it_alg = sum(r["alg_per_node"] for r in rows)
        record[key] = dict(kernels=rows, iteration_ms=it_ms, iteration_bytes_per_node=it_bytes,
                           iteration_alg_bytes_per_node=it_alg)
        md += [f"## {title}", "",
               "| kernel | role | working dispatches | avg ms | algorithmic B/node | HBM read B/node | "
               "HBM write B/node | measured GB/s | algorithmic GB/s |",
               "|---|---|---:|---:|---:|---:|---:|---:|---:|"]
        for r in rows:
            md.append(f"| {r['kernel']} | {r['role']} | {r['dispatches']} | {r['avg_ms']:.3f} | "
                      f"{r['alg_per_node']} | {r['read_per_node']:.1f} | {r['write_per_node']:.1f} | "
                      f"{r['gbs']:.0f} | {r['alg_gbs']:.0f} |")
        md += ["", f"One iteration: {it_ms:.3f} ms, {it_bytes:.1f} measured vs {it_alg} algorithmic HBM bytes per "
               f"fluid node ({it_alg * n_fluid / (it_ms * 1e-3) / 1e9:.0f} GB/s algorithmic).", ""]
        rounds = group(POT_ROUND_KERNELS) if key == "cg" else []
        if rounds:
            record["cg_round"] = dict(kernels=rounds)
            md += ["Once per refinement round:", "",
                   "| kernel | role | dispatches | avg ms | algorithmic B/node | HBM read B/node | "
                   "HBM write B/node | measured GB/s | algorithmic GB/s |",
                   "|---|---|---:|---:|---:|---:|---:|---:|---:|"]
            md += [f"| {r['kernel']} | {r['role']} | {r['dispatches']} | {r['avg_ms']:.3f} | {r['alg_per_node']} | "
                   f"{r['read_per_node']:.1f} | {r['write_per_node']:.1f} | {r['gbs']:.0f} | {r['alg_gbs']:.0f} |"
                   for r in rounds]
            md.append("")
    md += ["Commands (repository root; the three runs of the same bench command):", ""]
    md += [f"    {c}" for c in commands]
    return record, "\n".join(md) + "\n"


if __name__ == "__main__":
    main()
