"""Build libemin.so (HIP, gfx950) in-tree with hipcc.

Flags: -ffp-contract=off so every product and sum that decides an integer
(drop masks, Alg. 3 keys, Alg. 4 tests) is rounded separately; kernels that
want fused multiply-adds call fma() explicitly.  Packed FP32 instructions are
disabled (-packed-fp32-ops).
"""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libemin.so")
ARCH = os.environ.get("EMIN_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def build(verbose: bool = False, jobs: int = 8) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)
    flags = ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", "-I", os.path.join(ROOT, "include")]
    objs, procs = [], []
    for src in sources():
        obj = os.path.join(outdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc] + flags + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _drain(procs)
    _drain(procs)
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def _drain(procs):
    err = None
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            err = f"hipcc failed on {src}:\n{text}"
        elif text.strip():
            sys.stderr.write(text)
    procs.clear()
    if err:
        raise RuntimeError(err)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
