"""Build the gfx950 shared library ``libfunnel.so`` in-tree with hipcc.

Usage: python -m paper_1904_09409_amd.build   (or import and call build())"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "lib", "libfunnel.so")
SOURCES = ["funnel_kernels.hip", "funnel_peaks.hip", "funnel_api.cpp", "funnel_chirp.hip", "funnel_tables.cpp",
           "funnel_verify.hip", "funnel_refine.hip", "funnel_volume.hip", "funnel_queue.hip"] + [
    f"funnel_len_g{g}.hip" for g in range(6)] + [
    f"funnel_mfma_{p}_{g}.hip" for p in ("bf16", "fp16") for g in ("a", "b")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the exhaustive compile-time layout checks of the matrix-core engine
    "-fconstexpr-steps=200000000",
]


def _compile(src: str, obj: str) -> subprocess.Popen:
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    with tempfile.TemporaryDirectory() as tmp:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmp, src + ".o")
            objs.append(obj)
            procs.append((src, _compile(src, obj)))
        for src, p in procs:
            out, _ = p.communicate()
            out = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
            if p.returncode != 0:
                raise RuntimeError(f"hipcc failed on {src}:\n{out}")
            if verbose and out.strip():
                print(out)
        tmp_lib = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib, *objs]
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + r.stdout)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
