"""Build step of the HIP library: compiles csrc/ into liblbm.so for gfx950 with hipcc.

Each source is compiled to an object of its own (in parallel), then the objects are
linked into the shared library.  Every kernel is launched from the translation unit
that defines it, so no relocatable device code is needed."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["api.hip", "batch.hip", "kernels.hip", "adjoint.hip", "plan.cpp", "api3.hip",
           "kernels3.hip", "plan3.cpp", "noalloc.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")


def _flags() -> list[str]:
    return [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
            # packed FP32 instructions are kept out of all generated code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC,
            "-Wno-unused-command-line-argument"]


def hipcc_command(out: str) -> list[str]:
    """One hipcc call that compiles and links every source (the serial form)."""
    return ["hipcc", *_flags(), "-shared", *[os.path.join(CSRC, s) for s in SOURCES
                                              if os.path.exists(os.path.join(CSRC, s))],
            "-L", ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx", "-o", out]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 16))
    tmp = LIB + ".tmp%d" % os.getpid()
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as d:
        objs = [os.path.join(d, os.path.splitext(s)[0] + ".o") for s in srcs]

        def compile_one(k: int) -> None:
            cmd = ["hipcc", *_flags(), "-c", os.path.join(CSRC, srcs[k]), "-o", objs[k]]
            if verbose:
                print(" ".join(cmd), file=sys.stderr)
            subprocess.check_call(cmd)

        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(compile_one, range(len(srcs))))
        # The tracer's range API (rocprofiler-sdk-roctx) is linked with its path recorded.
        link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs,
                "-L", ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx", "-o", tmp]
        if verbose:
            print(" ".join(link), file=sys.stderr)
        subprocess.check_call(link)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
