"""Summaries of rocprofv3 output (rocpd SQLite databases) for the library's kernels.

    python -m paper_1307_4839_amd.rocprof_summary trace RESULTS.db [--skip NAME=K ...]

per kernel name: dispatch count, total and average duration over all
dispatches, and the average over the dispatches left after skipping the first
K dispatches of that kernel (``--skip``), e.g. the warmup steps of a benchmark
whose timed region starts after them.

    python -m paper_1307_4839_amd.rocprof_summary counters --fetch DB --write DB \\
        [--sq DB ...] --skip K --cells N --bytes1 B1 --bytes2 B2 --json OUT.json

    python -m paper_1307_4839_amd.rocprof_summary kernel --fetch DB --write DB \\
        --expect NAME=BYTES [...] --skip K --sources flowdir --json OUT.json

the same copy-calibrated FETCH_SIZE / WRITE_SIZE figures for the kernel
whose short name (template arguments included, parameters and namespaces
left out) is exactly NAME, e.g. 'flow_dir_kernel<float>', against BYTES
algorithmic bytes per launch; NAME#G restricts it to the dispatches whose
grid has G work-items along x (one launch shape of a kernel that runs on
several grids).  ``trace --by-grid`` splits the trace the same way.

For ``counters``, per stage kernel: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) averaged over
the dispatches after the first K, scaled by what the same counters read for
the plain device copy in the same runs (the largest __amd_rocclr_copyBuffer
dispatch, of known size 2^30 bytes each way), next to the algorithmic bytes
per launch (B1, B2 bytes per cell times N cells); with --sq, the SQ counters
of further runs (VALU and SALU instructions, waves, the VALU mix).  The JSON carries the
hash of the kernel sources so that a benchmark reads it only for the kernels
it was taken on.  ``--bench-log`` names the benchmark's stderr of one of
the runs: the simulated time and wet fraction at which its timed steps
started are recorded as the regime the counters describe.
"""

from __future__ import annotations

import argparse
import json
import sqlite3
import sys

COPY_BYTES = 1 << 30


def short_name(name: str) -> str:
    """Kernel name without 'void', namespaces and the parameter list."""
    return name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]


def regime_of(log: str) -> dict:
    """Simulated time and wet fraction when a benchmark's timed steps began,
    from its '[bench] spin-up ...' line."""
    import re
    with open(log) as f:
        for line in f:
            m = re.search(r"spin-up (\d+) \+ warmup (\d+) steps done, t = ([0-9.eE+-]+) s, "
                          r"wet fraction ([0-9.eE+-]+)", line)
            if m:
                return {"spinup_steps": int(m.group(1)), "warmup_steps": int(m.group(2)),
                        "t_start_s": float(m.group(3)), "wet_fraction": float(m.group(4))}
    raise SystemExit(f"{log}: no spin-up line")


def _stage(name: str) -> str | None:
    for s in ("1", "2"):
        if f"stage_kernel<{s}" in name:
            return f"stage_kernel<{s}>"
    return None


def _grids(con) -> dict:
    """{dispatch id: grid size along x}."""
    return dict(con.execute("select dispatch_id, grid_size_x from rocpd_kernel_dispatch"))


def trace(db: str, skip: dict, by_grid: bool = False) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, duration, dispatch_id from kernels "
                       "order by start").fetchall()
    grids = _grids(con) if by_grid else {}
    per = {}
    for name, start, dur, did in rows:
        short = short_name(name) + (f"#{grids.get(did, 0)}" if by_grid else "")
        per.setdefault(short, []).append(dur)
    out = []
    out.append(f"{'kernel':<60} {'calls':>6} {'total_ms':>10} {'avg_us':>10} "
               f"{'skip':>5} {'avg_us_after_skip':>18}")
    for name, durs in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        short = name
        k = 0
        for key, val in skip.items():
            if key in short:
                k = val
        rest = durs[k:] if k < len(durs) else []
        avg_rest = (sum(rest) / len(rest) / 1e3) if rest else float("nan")
        out.append(f"{short:<60} {len(durs):>6} {sum(durs) / 1e6:>10.3f} "
                   f"{sum(durs) / len(durs) / 1e3:>10.2f} {k:>5} {avg_rest:>18.2f}")
    return "\n".join(out)


def _counters(db: str, by_grid: bool = False):
    """{kernel name: [(dispatch id, {counter: value}), ...]} in dispatch order
    (with by_grid the key is 'name#grid size along x')."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, dispatch_id, counter_name, sum(counter_value) "
                       "from pmc_events group by dispatch_id, counter_name").fetchall()
    grids = _grids(con) if by_grid else {}
    per = {}
    for name, did, cn, v in rows:
        if by_grid:
            name = f"{name}#{grids.get(did, 0)}"
        per.setdefault(name, {}).setdefault(did, {})[cn] = v
    return {n: sorted(d.items()) for n, d in per.items()}


def _stage_avgs(db: str, skip: int):
    out = {}
    for name, disp in _counters(db).items():
        st = _stage(name)
        if st is None:
            continue
        rest = [c for _, c in disp[skip:]]
        if not rest:
            continue
        keys = set().union(*[c.keys() for c in rest])
        out[st] = {k: sum(c.get(k, 0.0) for c in rest) / len(rest) for k in keys}
        out[st]["_name"] = name
        out[st]["_dispatches"] = len(rest)
    return out


def _copy_counter(db: str, counter: str) -> float:
    best = 0.0
    for name, disp in _counters(db).items():
        if "copyBuffer" in name:
            for _, c in disp:
                best = max(best, c.get(counter, 0.0))
    if best <= 0.0:
        raise SystemExit(f"{db}: no copy dispatch with {counter} to calibrate against")
    return best


def counters(a) -> dict:
    from .build import source_hash
    fetch = _stage_avgs(a.fetch, a.skip)
    write = _stage_avgs(a.write, a.skip)
    cf = _copy_counter(a.fetch, "FETCH_SIZE")
    cw = _copy_counter(a.write, "WRITE_SIZE")
    ff = COPY_BYTES / 1024.0 / cf
    fw = COPY_BYTES / 1024.0 / cw
    # SQ counters of one or more runs (each run holds what one pass can
    # collect), merged per stage kernel
    sq = {}
    for db in a.sq or []:
        for st, vals in _stage_avgs(db, a.skip).items():
            sq.setdefault(st, {}).update(vals)
    rec = {"kernel_sha256_16": source_hash(), "workload": a.workload, "cells": a.cells,
           "regime": regime_of(a.bench_log) if a.bench_log else {},
           "calibration": {"probe": "1 GiB device-to-device copy (__amd_rocclr_copyBuffer)",
                           "fetch_KiB": cf, "write_KiB": cw,
                           "fetch_factor": ff, "write_factor": fw},
           "kernels": {}}
    for st, bpc in (("stage_kernel<1>", a.bytes1), ("stage_kernel<2>", a.bytes2)):
        if st not in fetch or st not in write:
            continue
        fk, wk = fetch[st]["FETCH_SIZE"], write[st]["WRITE_SIZE"]
        fb, wb = fk * 1024.0 * ff, wk * 1024.0 * fw
        alg = bpc * a.cells
        k = {"name": fetch[st]["_name"], "dispatches": fetch[st]["_dispatches"],
             "fetch_KiB_raw": fk, "write_KiB_raw": wk,
             "fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
             "algorithmic_bytes_per_launch": alg,
             "traffic_over_algorithmic": (fb + wb) / alg}
        if st in sq:
            k["sq"] = {kk: v for kk, v in sq[st].items() if not kk.startswith("_")}
        rec["kernels"][st] = k
    return rec


def kernel_counters(a) -> dict:
    from . import build
    paths = build.FLOWDIR_SOURCES if a.sources == "flowdir" else build.STAGE_SOURCES
    cf = _copy_counter(a.fetch, "FETCH_SIZE")
    cw = _copy_counter(a.write, "WRITE_SIZE")
    ff = COPY_BYTES / 1024.0 / cf
    fw = COPY_BYTES / 1024.0 / cw
    expect = {}
    for e in a.expect:
        k, v = e.rsplit("=", 1)
        expect[k] = int(v)
    by_grid = any("#" in k for k in expect)
    fetch, write = _counters(a.fetch, by_grid), _counters(a.write, by_grid)
    rec = {"kernel_sha256_16": build.source_hash(paths), "workload": a.workload,
           "calibration": {"probe": "1 GiB device-to-device copy (__amd_rocclr_copyBuffer)",
                           "fetch_KiB": cf, "write_KiB": cw,
                           "fetch_factor": ff, "write_factor": fw},
           "kernels": {}}
    for name in sorted(fetch):
        short = short_name(name)
        if by_grid:
            base, grid = name.rsplit("#", 1)
            short = short_name(base) + "#" + grid
        key = short if short in expect else None
        if key is None or name not in write:
            continue
        fr = [c["FETCH_SIZE"] for _, c in fetch[name][a.skip:] if "FETCH_SIZE" in c]
        wr = [c["WRITE_SIZE"] for _, c in write[name][a.skip:] if "WRITE_SIZE" in c]
        if not fr or not wr:
            continue
        fk, wk = sum(fr) / len(fr), sum(wr) / len(wr)
        fb, wb = fk * 1024.0 * ff, wk * 1024.0 * fw
        rec["kernels"][short] = {
            "name": name, "dispatches": len(fr), "fetch_KiB_raw": fk, "write_KiB_raw": wk,
            "fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
            "algorithmic_bytes_per_launch": expect[key],
            "traffic_over_algorithmic": (fb + wb) / expect[key]}
    return rec


def counters_text(rec: dict) -> str:
    c = rec["calibration"]
    out = []
    if rec.get("regime"):
        r = rec["regime"]
        out.append(f"regime: counters taken on steps from t = {r['t_start_s']:.2f} s, wet "
                   f"fraction {r['wet_fraction']:.4f} (after {r['spinup_steps']} spin-up + "
                   f"{r['warmup_steps']} warmup steps)")
    out += [f"calibration: the 1 GiB copy reads FETCH_SIZE = {c['fetch_KiB']:.0f} KiB and "
           f"WRITE_SIZE = {c['write_KiB']:.0f} KiB for 1048576 KiB moved each way: "
           f"fetch x{c['fetch_factor']:.4f}, write x{c['write_factor']:.4f}"]
    for st, k in rec["kernels"].items():
        out.append(f"{st:<16} FETCH {k['fetch_KiB_raw']:>12.0f} KiB ({k['fetch_bytes'] / 1e9:.3f} GB)"
                   f"  WRITE {k['write_KiB_raw']:>12.0f} KiB ({k['write_bytes'] / 1e9:.3f} GB)"
                   f"  total {k['bytes_per_launch'] / 1e9:.3f} GB  algorithmic "
                   f"{k['algorithmic_bytes_per_launch'] / 1e9:.3f} GB  ratio "
                   f"{k['traffic_over_algorithmic']:.3f}")
        if "sq" in k:
            sq = k["sq"]
            waves = sq.get("SQ_WAVES", 0.0)
            line = "   SQ: " + "  ".join(f"{kk}={v:.4g}" for kk, v in sorted(sq.items()))
            out.append(line)
            if "SQ_INSTS_VALU" in sq and rec["cells"]:
                per = 64.0 / rec["cells"]
                out.append(f"   VALU wave-instructions x 64 lanes per cell: "
                           f"{sq['SQ_INSTS_VALU'] * per:.1f}")
                kinds = [(kk[len("SQ_INSTS_VALU_"):], v) for kk, v in sorted(sq.items())
                         if kk.startswith("SQ_INSTS_VALU_")]
                if kinds:
                    out.append("   of which, per cell: " + "  ".join(
                        f"{kk} {v * per:.1f}" for kk, v in kinds))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--skip", action="append", default=[],
                   help="NAME=K: ignore the first K dispatches of kernels matching NAME")
    t.add_argument("--by-grid", action="store_true",
                   help="one line per kernel and grid size along x")
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--sq", action="append", default=[],
                   help="a run with SQ counters (repeatable: one per counter pass)")
    c.add_argument("--skip", type=int, default=0)
    c.add_argument("--cells", type=int, required=True)
    c.add_argument("--bytes1", type=int, required=True)
    c.add_argument("--bytes2", type=int, required=True)
    c.add_argument("--workload", default="")
    c.add_argument("--bench-log", help="the benchmark's stderr of one of the runs")
    c.add_argument("--json")
    k = sub.add_parser("kernel")
    k.add_argument("--fetch", required=True)
    k.add_argument("--write", required=True)
    k.add_argument("--expect", action="append", default=[],
                   help="NAME=BYTES: algorithmic bytes per launch of the kernel named NAME")
    k.add_argument("--skip", type=int, default=0)
    k.add_argument("--sources", choices=["stage", "flowdir"], default="stage")
    k.add_argument("--workload", default="")
    k.add_argument("--json")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        skip = {}
        for s in a.skip:
            k, v = s.rsplit("=", 1)
            skip[k] = int(v)
        print(trace(a.db, skip, a.by_grid))
        return 0
    rec = kernel_counters(a) if a.cmd == "kernel" else counters(a)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(rec, f, indent=1)
    print(counters_text(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
