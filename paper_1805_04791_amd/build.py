"""Builds libvie.so (HIP kernels + C++ runtime + C ABI) for gfx950 in-tree.

    python -m paper_1805_04791_amd.build [--jobs N] [--incremental]

Every source under csrc/ is compiled with hipcc to _build/*.o and linked into
paper_1805_04791_amd/libvie.so.  Packed-FP32 instructions are disabled for
all device code.
"""

from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libvie.so")

ARCH = os.environ.get("VIE_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def cflags():
    return ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC", "-x", "hip",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def sources():
    return [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith((".hip", ".cpp"))]


def headers():
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs.append(os.path.join(INCLUDE, "vie.h"))
    return hs


def _needs(src, obj, newest_header):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return os.path.getmtime(src) > t or newest_header > t


def _compile(src, obj):
    cmd = [hipcc()] + cflags() + ["-c", src, "-o", obj]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if p.returncode != 0:
        raise RuntimeError(f"compile failed: {os.path.basename(src)}\n{msgs}")
    return os.path.basename(src)


def build(jobs: int = 0, incremental: bool = False, verbose: bool = True) -> str:
    """Compile every source (only the out-of-date ones with `incremental`) and link."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in srcs]
    newest = max(os.path.getmtime(h) for h in headers())
    todo = [(s, o) for s, o in zip(srcs, objs) if not incremental or _needs(s, o, newest)]
    if jobs <= 0:
        jobs = min(16, max(1, len(os.sched_getaffinity(0))))
    if todo:
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            for name in ex.map(lambda so: _compile(*so), todo):
                if verbose:
                    print(f"  compiled {name}", flush=True)
    out = LIB
    tmp = out + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed\n" + p.stdout + p.stderr)
    os.replace(tmp, out)
    if verbose:
        print(f"  linked {out}", flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=0)
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args(argv)
    build(a.jobs, a.incremental)


if __name__ == "__main__":
    sys.exit(main())
