"""Compile the HIP library libmpts.so for gfx950 (in-tree).

The kernel source is compiled once per finalisation chunk size (CM = 4, 8,
16, 32; each compilation holds that instance of the forward and adjoint
kernels), the host code and the instance dispatch once each; the objects
build in parallel and are linked into one shared library.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpts.so")

CMS = (4, 8, 16, 32)

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _clean(text: str) -> str:
    return "\n".join(l for l in text.splitlines()
                     if "packed-fp32-ops" not in l and "unknown target feature" not in l
                     and l.strip() != "1 warning generated.")


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="mpts_build_") as tmp:
        jobs = []
        for cm in CMS:
            obj = os.path.join(tmp, f"kernels_cm{cm}.o")
            jobs.append((obj, [hipcc, *FLAGS, *inc, f"-DMPTS_CM={cm}", "-c",
                               os.path.join(CSRC, "mpts_kernels.hip"), "-o", obj]))
        for src in ("mpts_host.cpp", "mpts_dispatch.cpp", "mpts_probe.hip", "mpts_noalloc.hip"):
            obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
            jobs.append((obj, [hipcc, *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]))
        procs = []
        for obj, cmd in jobs:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
        errors = []
        for cmd, p in procs:
            out, _ = p.communicate()
            out = _clean(out)
            if p.returncode != 0:
                errors.append(" ".join(cmd) + "\n" + out)
            elif verbose and out.strip():
                print(out)
        if errors:
            raise RuntimeError("hipcc failed:\n" + "\n\n".join(errors))
        link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC",
                *[obj for obj, _ in jobs], "-o", LIB + ".tmp"]
        if verbose:
            print(" ".join(link), flush=True)
        r = subprocess.run(link, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed:\n" + _clean(r.stdout + r.stderr))
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
    sys.exit(0)
