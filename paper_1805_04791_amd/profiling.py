"""Summaries of rocprofv3 output for the solver's kernels.

    python -m paper_1805_04791_amd.profiling stats   --dir D --command CMD --out F.md [--top 16]
    python -m paper_1805_04791_amd.profiling traffic --fetch D1 --write D2 --kernel REGEX
           --command CMD --out F.md [--copy-regex REGEX --copy-bytes B]

``stats`` reads the ``*_kernel_stats.csv`` (``--stats``) and
``*_kernel_trace.csv`` (``--kernel-trace``) of one run: it lists rocprofv3's
own per-kernel statistics and, per kernel, the dispatches grouped by launch
shape (grid, workgroup), since the autotuner and the batch sizes of one run
launch the same kernel with different shapes.

``traffic`` reads two ``--pmc`` runs (``FETCH_SIZE``, then ``WRITE_SIZE``,
KiB per dispatch) and reports the HBM bytes per dispatch of the kernel
matching REGEX in its most frequent launch shape.  Each counter is scaled by
what it reads for a plain copy kernel of known size in the same run (the
dispatches matching --copy-regex, each moving --copy-bytes in and out).
The summary records the hash of the device sources that the profiled run
printed (``source_digest`` of its bench JSON line), so that a reader can
tell whether the kernels changed since the counters were taken.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import statistics
import sys
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# headers holding device code (the others declare host interfaces)
DEVICE_HEADERS = ("cx.hpp", "dft.hpp", "fft.hpp", "apply_kernels.hpp", "lens.hpp", "symbol.hpp")


def source_digest() -> str:
    """sha256 over the sources the apply kernels are compiled from (the shared
    device headers and the per-length files; names and contents, sorted)."""
    h = hashlib.sha256()
    paths = [os.path.join(CSRC, f) for f in DEVICE_HEADERS] + glob.glob(os.path.join(CSRC, "len_*.hip"))
    for path in sorted(paths):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    """'void vie::k_zpass<float, 16, 16, 3, 0>(...)' -> 'k_zpass<float, 16, 16, 3, 0>'."""
    n = name.replace("vie::(anonymous namespace)::", "").replace("vie::", "")
    n = re.sub(r"^void ", "", n)
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return n[:i]
    return n


def read_stats(d: str):
    rows = []
    with open(_find(d, "kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]),
                         float(r["AverageNs"]), float(r["Percentage"])))
    return rows


def _find(d: str, suffix: str) -> str:
    for root, _, files in os.walk(d):
        for fn in sorted(files):
            if fn.endswith(suffix):
                return os.path.join(root, fn)
    raise FileNotFoundError(f"no *{suffix} under {d}")


def read_trace(d: str):
    """{kernel: {(grid_items, wg): [durations in ns]}}"""
    out = defaultdict(lambda: defaultdict(list))
    with open(_find(d, "kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            out[short_name(r["Kernel_Name"])][(grid, wg)].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def stats_summary(d: str, command: str, top: int = 16, bench: dict = None) -> str:
    rows = read_stats(d)
    trace = read_trace(d)
    digest = bench["roofline"]["source_digest"] if bench else source_digest()
    lines = ["# rocprofv3 kernel statistics", "", "Command (`$REPO` = the repository root; one MI355X):", "",
             "```", command, "```", "",
             f"Device sources of the profiled run: `source_digest = {digest}`", ""]
    if bench:
        roof = bench["roofline"]
        lines += [f"The run's own HIP-event timing of its dominant kernel family `{roof['kernel']}`: "
                  f"{roof['avg_launch_us']:.1f} us per launch over its profiled pass "
                  f"(value {bench['value']:.2f} {bench['unit']}, from the timed steps).", ""]
    lines += [
              "## rocprofv3 --stats (all dispatches of the run)", "",
              "| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in sorted(rows, key=lambda r: -r[2])[:top]:
        lines.append(f"| `{name}` | {calls} | {tot / 1e6:.2f} | {avg / 1e3:.1f} | {pct:.2f} |")
    lines += ["", "## Dispatches by launch shape (kernel trace)", "",
              "Shapes with at least 4 dispatches of the kernels above; grid in work-items.", "",
              "| kernel | grid | workgroup | dispatches | avg us | median us |", "|---|---|---|---|---|---|"]
    names = [r[0] for r in sorted(rows, key=lambda r: -r[2])[:top]]
    for name in names:
        for (grid, wg), durs in sorted(trace.get(name, {}).items(), key=lambda kv: -len(kv[1])):
            if len(durs) < 4:
                continue
            lines.append(f"| `{name}` | {grid} | {wg} | {len(durs)} | {statistics.mean(durs) / 1e3:.1f} | "
                         f"{statistics.median(durs) / 1e3:.1f} |")
    return "\n".join(lines) + "\n"


def read_counters(d: str, counter: str):
    """{kernel: {(grid_items, wg): [values]}} for one counter."""
    out = defaultdict(lambda: defaultdict(list))
    with open(_find(d, "counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            out[short_name(r["Kernel_Name"])][(int(r["Grid_Size"]), int(r["Workgroup_Size"]))].append(
                float(r["Counter_Value"]))
    return out


def _pick(groups: dict, regex: str):
    rx = re.compile(regex)
    cands = [(k, shape, v) for k, shapes in groups.items() if rx.search(k) for shape, v in shapes.items()]
    if not cands:
        raise KeyError(f"no kernel matches {regex!r}")
    return max(cands, key=lambda c: len(c[2]))


def traffic_summary(fetch_dir: str, write_dir: str, kernel: str, command: str, copy_regex: str,
                    copy_bytes: float, algorithmic: float = None, digest: str = None) -> str:
    digest = digest or source_digest()
    fetch = read_counters(fetch_dir, "FETCH_SIZE")
    write = read_counters(write_dir, "WRITE_SIZE")
    kname, shape, fv = _pick(fetch, kernel)
    wv = write[kname][shape]
    # calibration: the copy dispatches that moved copy_bytes
    _, cshape, cf = _pick(fetch, copy_regex)
    cw = write[_pick(write, copy_regex)[0]][cshape]
    f_copy = statistics.median(cf) * 1024.0
    w_copy = statistics.median(cw) * 1024.0
    f_scale = copy_bytes / f_copy
    w_scale = copy_bytes / w_copy
    f_k = statistics.mean(fv) * 1024.0 * f_scale
    w_k = statistics.mean(wv) * 1024.0 * w_scale
    lines = ["# HBM traffic per dispatch (rocprofv3 --pmc)", "", "Commands (`$REPO` = the repository root; one MI355X):",
             "", "```", command, "```", "",
             f"Device sources of the profiled runs: `source_digest = {digest}`", "",
             f"Kernel: `{kname}`, launch shape grid {shape[0]} work-items, workgroup {shape[1]} "
             f"({len(fv)} FETCH / {len(wv)} WRITE dispatches).", "",
             "| quantity | value |", "|---|---|",
             f"| FETCH_SIZE per dispatch (raw) | {statistics.mean(fv):.1f} KiB |",
             f"| WRITE_SIZE per dispatch (raw) | {statistics.mean(wv):.1f} KiB |",
             f"| copy calibration: {copy_bytes / 2**20:.0f} MiB read + written | FETCH {statistics.median(cf):.1f} KiB, "
             f"WRITE {statistics.median(cw):.1f} KiB |",
             f"| scale factors | FETCH x{f_scale:.3f}, WRITE x{w_scale:.3f} |",
             f"| fetched bytes per dispatch (scaled) | {f_k:.4g} |",
             f"| written bytes per dispatch (scaled) | {w_k:.4g} |",
             f"| traffic per dispatch | {f_k + w_k:.4g} |"]
    if algorithmic:
        lines.append(f"| algorithmic bytes per dispatch | {algorithmic:.4g} (traffic / algorithmic = "
                     f"{(f_k + w_k) / algorithmic:.3f}) |")
    lines += ["", f"traffic_bytes_per_launch: {f_k + w_k:.6g}", f"kernel: {kname}",
              f"source_digest: {digest}", ""]
    return "\n".join(lines)


def read_traffic(path: str):
    """(traffic bytes per launch, kernel, digest) from a traffic summary, or None."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^(traffic_bytes_per_launch|kernel|source_digest): (.+)$", line.strip())
            if m:
                vals[m.group(1)] = m.group(2)
    if len(vals) < 3:
        return None
    return float(vals["traffic_bytes_per_launch"]), vals["kernel"], vals["source_digest"]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--dir", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--top", type=int, default=16)
    s.add_argument("--bench-json", default=None, help="stdout of the profiled bench run")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--copy-regex", default=r"vectorized_elementwise_kernel|elementwise_kernel")
    t.add_argument("--copy-bytes", type=float, default=float(2**30))
    t.add_argument("--algorithmic", type=float, default=None)
    t.add_argument("--bench-json", default=None,
                   help="stdout of the profiled bench run: source digest and algorithmic bytes per launch")
    a = ap.parse_args(argv)
    if a.what == "stats":
        bench = None
        if a.bench_json:
            import json
            with open(a.bench_json) as f:
                bench = json.loads(f.read().strip().splitlines()[-1])
        text = stats_summary(a.dir, a.command, a.top, bench)
    else:
        digest, alg = None, a.algorithmic
        if a.bench_json:
            import json
            with open(a.bench_json) as f:
                roof = json.loads(f.read().strip().splitlines()[-1])["roofline"]
            digest = roof["source_digest"]
            alg = alg or roof["bytes_per_launch"]
        text = traffic_summary(a.fetch, a.write, a.kernel, a.command, a.copy_regex, a.copy_bytes, alg, digest)
    with open(a.out, "w") as f:
        f.write(text)
    print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
