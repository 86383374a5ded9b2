"""Build libsylv.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2204_08057_amd.build          # or: python paper_2204_08057_amd/build.py

The library is written next to this file so it travels with the source tree.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libsylv.so")
# longest compile first: the instantiations of the block solver (per right-hand-side count and
# precision) and of the Fourier preconditioner's passes (per precision and grid type)
SOURCES = ["sylv_block_s8_f32.hip", "sylv_block_s8_f64.hip", "sylv_block_s4_f32.hip",
           "sylv_kernels.hip", "sylv_fourier_f64_periodic.hip", "sylv_fourier_f64_face.hip",
           "sylv_block_s4_f64.hip", "sylv_fourier_f32_periodic.hip", "sylv_fourier_f32_face.hip",
           "sylv_block_s2_f32.hip", "sylv_block_s2_f64.hip", "sylv_lanczos.hip", "sylv_block.hip",
           "sylv_kohler.hip", "sylv_fourier.hip", "sylv_api.hip"]
ARCH = os.environ.get("SYLV_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm toolchain required to build libsylv)")


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # never emit packed fp32 VALU instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
        f"-I{INCLUDE}", f"-I{CSRC}",
    ]


def build(verbose: bool = True, jobs: int = 0) -> str:
    """Compile every source to an object in a temp dir (jobs at a time, default one per CPU up
    to 8), then link the shared library."""
    cc = hipcc()
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    tmp = tempfile.mkdtemp(prefix="sylv_build_")
    try:
        objs = [os.path.join(tmp, src.replace(".hip", ".o")) for src in SOURCES]

        def compile_one(src, obj):
            cmd = [cc, *flags(), "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            return src, subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                       text=True)

        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
            for src, proc in pool.map(compile_one, SOURCES, objs):
                _check(src, proc, verbose)
        out_tmp = LIB + ".tmp"
        cmd = [cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", out_tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


def _check(src, proc, verbose):
    msgs = [ln for ln in proc.stdout.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout)
        raise RuntimeError(f"hipcc failed on {src}")
    if verbose and msgs:
        print("\n".join(msgs))


if __name__ == "__main__":
    print(build())
