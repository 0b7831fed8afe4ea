"""Build liblbm.so for gfx950 with hipcc (in-tree, next to this file).

Run as ``python paper_1507_06767_amd/build.py`` (by path: importing the
package would load the library being rebuilt).  The host runtime and the
step-kernel instantiations of each storage family are separate translation
units, compiled in parallel and linked into one shared library.  Flags: -O3,
C++20, no fast-math (division and square root stay correctly rounded), and
the packed FP32 instructions disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["lbm.hip", "step_f64.hip", "step_f32.hip", "step_f16.hip", "step_bf16.hip", "cnn.hip"]
OUT = os.path.join(HERE, "liblbm.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(out: str = OUT, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmp:
        objs = [os.path.join(tmp, src.replace(".hip", ".o")) for src in SOURCES]

        def compile_one(k):
            cmd = [hipcc, *HIPCC_FLAGS, *extra, "-c", "-o", objs[k], os.path.join(CSRC, SOURCES[k])]
            return subprocess.run(cmd).returncode

        with ThreadPoolExecutor(max_workers=jobs) as pool:
            codes = list(pool.map(compile_one, range(len(SOURCES))))
        failed = [src for src, rc in zip(SOURCES, codes) if rc != 0]
        if failed:
            raise RuntimeError(f"hipcc failed for {failed}")
        tmp_out = out + ".tmp"
        subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_out, *objs],
                       check=True)
        os.replace(tmp_out, out)
    return out


if __name__ == "__main__":
    print(build(extra=sys.argv[1:]))
