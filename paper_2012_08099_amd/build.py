"""Build libdpm.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2012_08099_amd.build [--jobs N]

Every HIP source is compiled for gfx950 only, with packed FP32 instructions disabled,
then linked into ``paper_2012_08099_amd/libdpm.so``.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdpm.so")
SOURCES = [
    "slice_g0_u16_fast.hip", "slice_g0_u16_gen.hip", "slice_g0_u8_fast.hip", "slice_g0_u8_gen.hip",
    "slice_g12_u16.hip", "slice_g12_u8.hip", "slice_groups_u16.hip", "slice_groups_u8.hip",
    "slice_batched.hip", "slice_block_u8.hip", "slice_block_u16.hip", "power_kernels.hip", "features.hip", "from_images.hip",
    "moment_kernels.hip", "noalloc.hip", "paper_mode.hip", "paper_api.cpp", "resident.hip", "slice_dispatch.cpp", "dpm_api.cpp", "batched.cpp", "server.cpp",
]
ARCH = "gfx950"


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def common_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
        "-Wno-unused-function", "-Wno-unused-variable",
        # packed FP32 instructions stay off (device pass; the host pass ignores it)
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(HERE, "..", "include"), "-I", CSRC,
    ]


def _includes(path, seen):
    """The quoted #include files a source pulls in, recursively (csrc/ and include/)."""
    import re
    with open(path) as fh:
        for line in fh:
            m = re.match(r'\s*#include\s+"([^"]+)"', line)
            if not m:
                continue
            dep = os.path.normpath(os.path.join(os.path.dirname(path), m.group(1)))
            if dep not in seen and os.path.exists(dep):
                seen.add(dep)
                _includes(dep, seen)
    return seen


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    path = os.path.join(CSRC, src)
    deps = [path] + sorted(_includes(path, set()))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def compile_one(src, force=True):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if not force and not _stale(src, obj):
        return obj, ""
    cmd = [hipcc()] + common_flags() + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{out}")
    return obj, out


def build(jobs=None, verbose=False, force=True):
    """Compile every source (``force=False``: only stale objects) and link libdpm.so."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: compile_one(s, force), SOURCES))
    if verbose:
        for _, out in results:
            if out.strip():
                print(out)
    objs = [o for o, _ in results]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--incremental", action="store_true", help="recompile stale objects only")
    a = ap.parse_args(argv)
    print(build(a.jobs, a.verbose, force=not a.incremental))


if __name__ == "__main__":
    sys.exit(main())
