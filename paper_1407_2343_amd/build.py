"""Builds libsnlm.so for gfx950 in-tree.

Every kernel variant for one search half-width S lives in its own translation
unit (snlm_inst.hip compiled with -DSNLM_S=<S>), so the 17 units compile in
parallel; the host library (snlm_api.cpp) is compiled with hipcc and the whole
is linked into paper_1407_2343_amd/libsnlm.so.

    python -m paper_1407_2343_amd.build [--jobs N] [--only-s 5,10,15] [--incremental]

``--only-s`` restricts the compiled S values (the others are then missing from
the library and rejected at run time); it is for quick development builds.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsnlm.so")
ARCH = "gfx950"

# -packed-fp32-ops: no packed FP32 instructions (v_pk_*_f32) anywhere.
# -ffp-contract=off: only the fused multiply-adds written in the source, so every
# code path (pre-chunk, main chunk, any segment length) rounds identically.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off"]
COMMON = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall"]


def _run(cmd):
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l and "hip-link" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return time.time() - t0, out


def _fresh(obj, deps):
    """True when obj exists and is newer than every dependency."""
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps)


def build(jobs: int | None = None, only_s=None, verbose: bool = False, incremental: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or int(os.environ.get("SNLM_BUILD_JOBS", "0")) or max(1, os.cpu_count() or 1)
    s_values = list(range(0, 17)) if only_s is None else sorted(set([0] + list(only_s)))
    objs, cmds = [], []
    # what snlm_inst.hip includes (snlm_issue.hip is a unit of its own)
    dev_deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hpp") or f == "snlm_inst.hip"]
    for s in s_values:
        o = os.path.join(BUILD, "snlm_inst_s%d.o" % s)
        objs.append(o)
        if incremental and _fresh(o, dev_deps + [os.path.abspath(__file__)]):
            continue
        cmds.append(COMMON + DEVICE_FLAGS + ["-DSNLM_S=%d" % s, "-c",
                                            os.path.join(CSRC, "snlm_inst.hip"), "-o", o])
    api_o = os.path.join(BUILD, "snlm_api.o")
    objs.append(api_o)
    cmds.append(COMMON + DEVICE_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, "snlm_api.cpp"),
                                        "-o", api_o])
    issue_o = os.path.join(BUILD, "snlm_issue.o")
    objs.append(issue_o)
    cmds.append(COMMON + DEVICE_FLAGS + ["-c", os.path.join(CSRC, "snlm_issue.hip"), "-o", issue_o])
    stubs = None
    if only_s is not None:
        # empty registration functions for the S values left out
        missing = [s for s in range(17) if s not in s_values]
        stubs = os.path.join(BUILD, "snlm_stubs.cpp")
        with open(stubs, "w") as f:
            f.write('#include "snlm_registry.hpp"\nextern "C" {\n')
            for s in missing:
                f.write("void snlm_register_s%d(snlm::KernelRegistry*) {}\n" % s)
            f.write("}\n")
        so = os.path.join(BUILD, "snlm_stubs.o")
        objs.append(so)
        cmds.append(COMMON + ["-x", "hip", "-c", stubs, "-o", so])
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for (dt, out), cmd in zip(ex.map(_run, cmds), cmds):
            if verbose:
                print("%6.1fs %s" % (dt, cmd[-1]), flush=True)
            if out.strip() and verbose:
                print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0), flush=True)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--only-s", type=str, default=None)
    ap.add_argument("--incremental", action="store_true",
                    help="reuse kernel objects newer than the kernel sources")
    a = ap.parse_args(argv)
    only = [int(v) for v in a.only_s.split(",")] if a.only_s else None
    build(a.jobs, only, verbose=True, incremental=a.incremental)


if __name__ == "__main__":
    sys.exit(main())
