"""Build liblbm.so for gfx950 with hipcc (in-tree, next to this file).

Run as ``python paper_1507_06767_amd/build.py`` (by path: importing the
package would load the library being rebuilt).  The host runtime, the
predictor kernels, one object per step-kernel instantiation (lattice x
storage type, all from step_inst.hip) and the patch-hierarchy kernels per
lattice and storage family (patch_inst.hip) are compiled in parallel and linked into one shared
library.  Flags: -O3, C++20, no fast-math (division and
square root stay correctly rounded), multiply-adds fused only within one
source expression (-ffp-contract=on: kernels that spell the same arithmetic
round the same way, whatever code surrounds it), and the packed FP32
instructions disabled for the device code.
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
LATTICES = (9, 19, 27)
# storage type, arithmetic type, shifted storage, object tag
STORAGE_TYPES = [("double", "double", "false", "f64"), ("float", "float", "false", "f32"),
                 ("float", "float", "true", "f32s"), ("_Float16", "float", "true", "f16s"),
                 ("half_sr", "float", "true", "f16sr"), ("__bf16", "float", "true", "bf16s"),
                 ("bf16_sr", "float", "true", "bf16sr")]
# (source, extra defines, object name)
UNITS = [("lbm.hip", [], "lbm.o"), ("cnn.hip", [], "cnn.o")] + [
    ("step_inst.hip", [f"-DLBM_Q={q}", f"-DLBM_T={t}", f"-DLBM_C={c}", f"-DLBM_SH={sh}"], f"step_q{q}_{tag}.o")
    for q in LATTICES for t, c, sh, tag in STORAGE_TYPES] + [
    ("patch_inst.hip", [f"-DLBM_Q={q}", f"-DLBM_PATCH_SET={ps}"], f"patch_q{q}_{ps}.o")
    for q in (19, 27) for ps in (0, 1)]
SOURCES = sorted({u[0] for u in UNITS})
OUT = os.path.join(HERE, "liblbm.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def build(out: str = OUT, extra=()) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = max(1, min(len(UNITS), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with tempfile.TemporaryDirectory(prefix="lbm_build_") as tmp:
        objs = [os.path.join(tmp, u[2]) for u in UNITS]

        def compile_one(k):
            src, defines, _ = UNITS[k]
            cmd = [hipcc, *HIPCC_FLAGS, *defines, *extra, "-c", "-o", objs[k], os.path.join(CSRC, src)]
            return subprocess.run(cmd).returncode

        # the largest units first, so that they do not start last
        order = sorted(range(len(UNITS)), key=lambda k: UNITS[k][0] == "cnn.hip")
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            codes = dict(zip(order, pool.map(compile_one, order)))
        failed = [UNITS[k][2] for k in range(len(UNITS)) if codes[k] != 0]
        if failed:
            raise RuntimeError(f"hipcc failed for {failed}")
        tmp_out = out + ".tmp"
        subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_out, *objs],
                       check=True)
        os.replace(tmp_out, out)
    return out


if __name__ == "__main__":
    print(build(extra=sys.argv[1:]))
