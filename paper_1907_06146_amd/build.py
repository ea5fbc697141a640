"""Compile libssg.so for gfx950 with hipcc (in-tree): every source is
compiled to an object in parallel, then the objects are linked."""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", n) for n in
           ("ssg_search.hip", "ssg_groups.hip", "ssg_knn.hip", "ssg_build.hip", "ssg_merge.hip")]
OUT = os.path.join(HERE, "libssg.so")
OBJ_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    tag = f".{os.getpid()}"
    objs = [os.path.join(OBJ_DIR, os.path.basename(s) + tag + ".o") for s in SOURCES]
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = [ex.submit(_run, [HIPCC] + FLAGS + ["-c", s, "-o", o], verbose)
                for s, o in zip(SOURCES, objs)]
        for f in futs:
            f.result()
    tmp = OUT + f".tmp{os.getpid()}"
    try:
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
        os.replace(tmp, OUT)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
