"""Build libqqa.so (HIP kernels + host runtime + C ABI) in-tree for gfx950 with hipcc."""

from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys
import tempfile

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libqqa.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["qqa_kernels.hip", "qqa_scratch.hip", "qqa_slots.hip", "qqa_persist.hip", "qqa_dense.hip", "qqa_color.hip", "qqa_slice.hip", "qqa_compact.hip", "qqa_resident.hip", "qqa_runtime.cpp", "qqa_ctx.cpp", "qqa_serve.cpp", "qqa_server.cpp"]
HEADERS = ["qqa_internal.h", "qqa_runtime.h", "qqa_ctx.h", "qqa_device.h", "qqa_batch.h"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    "-mcode-object-version=5",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # explicit fmaf only: identical rounding in every kernel that shares a device function
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result",
]


def sources() -> list[str]:
    return [os.path.join(CSRC, s) for s in SOURCES]


def _run(cmd: list[str], verbose: bool) -> None:
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libqqa.so")
    if verbose and r.stderr.strip():
        # hipcc's host pass does not know the gfx feature flag; everything else is shown
        lines = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every HIP/C++ source (in parallel, one object each) and link one shared
    library next to this file."""
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 1, 16))
    with tempfile.TemporaryDirectory(prefix="qqa_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in sources()]
        cmds = [[HIPCC, *compile_flags, *inc, "-c", src, "-o", obj] for src, obj in zip(sources(), objs)]
        with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
            for f in [pool.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp%d" % os.getpid()
        _run([HIPCC, *FLAGS, *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "qqa.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    print(build(verbose=True))
