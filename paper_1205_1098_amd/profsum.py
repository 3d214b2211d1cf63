"""Summaries of rocprofv3 runs for the profiles/ directory.

  python -m paper_1205_1098_amd.profsum trace DB --label L --command CMD --out FILE
      per-kernel dispatch statistics of a --kernel-trace run
  python -m paper_1205_1098_amd.profsum counters --fetch DB --write DB --copy-fetch DB
      --copy-write DB --kernel SUBSTR --label L --alg-bytes B --command CMD --out FILE
      HBM bytes per dispatch of one kernel from two --pmc runs (FETCH_SIZE, then
      WRITE_SIZE), each scaled by what the same counter reads for the 2 GiB copy
      probe, whose bytes are known; with --unit SUBSTR, the bytes of every
      dispatch matching --kernel per dispatch matching SUBSTR (the launches of
      a plan made of several kernels)

The counter summary records the digest of the kernel sources; the benchmark
only reports its traffic while the sources still match.
"""

from __future__ import annotations

import argparse
import hashlib
import os
import sqlite3
import statistics

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# what defines a measured kernel: its device code, the shared device helpers
# and launch declarations, and (matrix sweeps) the tuned configurations
SOURCE_SETS = {
    "matrix": ["paper_1205_1098_amd/csrc/bto_mat.hip", "paper_1205_1098_amd/csrc/bto_tile.hpp",
               "paper_1205_1098_amd/csrc/bto_dev.hpp",
               "paper_1205_1098_amd/csrc/bto_internal.hpp", "paper_1205_1098_amd/csrc/bto_tuned.hpp"],
    "tiled": ["paper_1205_1098_amd/csrc/bto_btile.hip", "paper_1205_1098_amd/csrc/bto_tile.hpp",
              "paper_1205_1098_amd/csrc/bto_dev.hpp", "paper_1205_1098_amd/csrc/bto_internal.hpp",
              "paper_1205_1098_amd/csrc/bto_api.hip"],
    "vector": ["paper_1205_1098_amd/csrc/bto_vec.hip", "paper_1205_1098_amd/csrc/bto_dev.hpp",
               "paper_1205_1098_amd/csrc/bto_internal.hpp"],
    "batch": ["paper_1205_1098_amd/csrc/bto_batch.hip", "paper_1205_1098_amd/csrc/bto_batch.hpp",
              "paper_1205_1098_amd/csrc/bto_dev.hpp", "paper_1205_1098_amd/csrc/bto_internal.hpp"],
}
COPY_BYTES = (1 << 28) * 8      # the copy probe reads and writes 2 GiB per launch


def source_digest(source_set: str = "matrix") -> str:
    h = hashlib.sha256()
    for rel in SOURCE_SETS[source_set]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _dispatches(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration from kernels").fetchall()
    con.close()
    return rows


def _pmc(db: str, counter: str):
    con = sqlite3.connect(db)
    rows = con.execute("select name, counter_value from pmc_events where counter_name = ?",
                       (counter,)).fetchall()
    con.close()
    return rows


def trace_summary(db: str, label: str, command: str) -> str:
    by = {}
    for name, dur in _dispatches(db):
        by.setdefault(name, []).append(dur)
    total = sum(sum(v) for v in by.values()) or 1
    lines = [f"# rocprofv3 kernel trace: {label}", "", "Command:", "", "    " + command, "",
             "| kernel | calls | total ms | avg us | min us | max us | % time |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for name, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{name}` | {len(v)} | {sum(v) / 1e6:.3f} | {statistics.mean(v) / 1e3:.2f} "
                     f"| {min(v) / 1e3:.2f} | {max(v) / 1e3:.2f} | {100 * sum(v) / total:.1f} |")
    return "\n".join(lines) + "\n"


def counters_summary(fetch: str, write: str, cfetch: str, cwrite: str, kernel: str,
                     label: str, alg_bytes: float, command: str, sources: str = "matrix",
                     unit: str | None = None) -> str:
    """Without `unit`: the median per dispatch of the kernels matching
    `kernel`.  With it: every dispatch matching `kernel` summed and divided
    by the number of dispatches matching `unit` (one per launch of a
    multi-kernel plan), with a per-kernel breakdown."""
    def per_dispatch(rows, sub, unit=None):
        vals = [v for name, v in rows if sub in name]
        if not vals:
            raise SystemExit(f"no dispatch of a kernel matching {sub!r}")
        if unit is None:
            return statistics.median(vals), len(vals)
        units = sum(1 for name, _ in rows if unit in name)
        if not units:
            raise SystemExit(f"no dispatch of a kernel matching {unit!r}")
        return sum(vals) / units, units

    cf, _ = per_dispatch(_pmc(cfetch, "FETCH_SIZE"), "k_copy")
    cw, _ = per_dispatch(_pmc(cwrite, "WRITE_SIZE"), "k_copy")
    f_factor = COPY_BYTES / (cf * 1024.0)
    w_factor = COPY_BYTES / (cw * 1024.0)
    kf, nf = per_dispatch(_pmc(fetch, "FETCH_SIZE"), kernel, unit)
    kw, nw = per_dispatch(_pmc(write, "WRITE_SIZE"), kernel, unit)
    fb, wb = kf * 1024.0 * f_factor, kw * 1024.0 * w_factor
    breakdown = []
    if unit is not None:
        fr, wr = _pmc(fetch, "FETCH_SIZE"), _pmc(write, "WRITE_SIZE")
        names = sorted({name for name, _ in fr if kernel in name})
        breakdown = ["", f"per launch (dispatches matching {kernel!r} per dispatch of {unit!r}):", ""]
        for nm in names:
            f1 = sum(v for n_, v in fr if n_ == nm) / nf * 1024.0 * f_factor
            w1 = sum(v for n_, v in wr if n_ == nm) / nw * 1024.0 * w_factor
            short = nm.replace("bto::(anonymous namespace)::", "").replace("void ", "")
            short = short.split("(")[0]
            breakdown.append(f"    {short}: {f1 / 1e9:.3f} GB fetched + {w1 / 1e9:.3f} GB written")
        breakdown.append("")
    lines = [
        f"# HBM traffic per dispatch: {label}",
        "",
        "Commands (each rocprofv3 --pmc pass is its own run):",
        "",
        *("    " + c for c in command.split(" ;; ")),
        "",
        *breakdown,
        f"kernel: {kernel}",
        *([f"per_launch_of: {unit}"] if unit is not None else []),
        f"{'launches' if unit is not None else 'dispatches'}_measured: {nf} (FETCH_SIZE), "
        f"{nw} (WRITE_SIZE)",
        f"copy_probe_bytes: {COPY_BYTES}",
        f"copy_fetch_kib: {cf:.3f}",
        f"copy_write_kib: {cw:.3f}",
        f"fetch_factor: {f_factor:.5f}",
        f"write_factor: {w_factor:.5f}",
        f"kernel_fetch_kib: {kf:.3f}",
        f"kernel_write_kib: {kw:.3f}",
        f"hbm_fetch_bytes: {fb:.0f}",
        f"hbm_write_bytes: {wb:.0f}",
        f"hbm_bytes_per_launch: {fb + wb:.0f}",
        f"alg_bytes_per_launch: {alg_bytes:.0f}",
        f"amplification: {(fb + wb) / alg_bytes:.4f}",
        f"source_set: {sources}",
        f"source_digest: {source_digest(sources)}",
    ]
    return "\n".join(lines) + "\n"


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    c = sub.add_parser("counters")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--kernel"):
        c.add_argument(a, required=True)
    c.add_argument("--alg-bytes", type=float, required=True)
    c.add_argument("--unit", default=None,
                   help="sum the --kernel dispatches per dispatch of this kernel (one per "
                        "launch of a multi-kernel plan)")
    c.add_argument("--sources", choices=sorted(SOURCE_SETS), default="matrix",
                   help="the source set whose digest the summary records")
    for p in (t, c):
        p.add_argument("--label", required=True)
        p.add_argument("--command", required=True)
        p.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    if args.cmd == "trace":
        text = trace_summary(args.db, args.label, args.command)
    else:
        text = counters_summary(args.fetch, args.write, args.copy_fetch, args.copy_write,
                                args.kernel, args.label, args.alg_bytes, args.command,
                                args.sources, args.unit)
    with open(args.out, "w") as f:
        f.write(text)
    print(text)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
