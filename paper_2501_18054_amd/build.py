"""Builds libpngf.so in-tree with hipcc for gfx950.

    python -m paper_2501_18054_amd.build   (or build() from Python)
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpngf.so")
SOURCES = ["host_precompute.cpp", "pngf_api.hip", "plain_kernels.hip", "lu_kernels.hip", "mixed_kernels.hip", "step_kernels.hip", "cnn.hip", "gemm_kernels.hip", "tile_kernels.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose=False):
    objs = []
    jobs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        # host C++ (the precompute): AVX2 + FMA, present on every x86-64 host
        # of these GPUs; its GEMM kernel is written with those intrinsics
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-mavx2", "-mfma"]
        cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-fopenmp",
               "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument",
               "-I", os.path.join(HERE, "..", "include"), "-c"] + lang + [path, "-o", obj]
        jobs.append((src, cmd))
        objs.append(obj)
    procs = [(src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
             for src, cmd in jobs]
    for src, cmd, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the packed-fp32 target feature: harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            sys.stderr.write(text)
            raise RuntimeError(f"hipcc failed on {src}")
        if verbose and lines:
            print("\n".join(lines))
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-fopenmp", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        sys.stderr.write(r.stdout.decode(errors="replace"))
        raise RuntimeError("link of libpngf.so failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
