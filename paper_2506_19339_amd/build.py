"""Build libctm.so (and the kernel self-test library) for gfx950 with hipcc.

Usage: python -m paper_2506_19339_amd.build   (or __graft_entry__.build())
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "--offload-arch=" + ARCH,
    # no packed FP32 instructions in any HIP code: some of their forms have
    # given wrong results on gfx950 without any error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]

TARGETS = {
    "libctm.so": ["kernels.hip", "engine.hip"],
    "libctm_selftest.so": ["kernels.hip", "selftest.hip"],
}


def build(verbose=False):
    for lib, srcs in TARGETS.items():
        out = os.path.join(HERE, lib)
        tmp = out + ".tmp"
        cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in srcs] + ["-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed for %s" % lib)
        os.replace(tmp, out)
    return os.path.join(HERE, "libctm.so")


if __name__ == "__main__":
    print(build(verbose=True))
