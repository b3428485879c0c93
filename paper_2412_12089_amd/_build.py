"""Builds the HIP library libmpmx.so in place with hipcc for gfx950."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmpmx.so")
SOURCES = ["mpm_kernels.hip", "mpm_kernels_lds.hip", "mpm_observe.hip", "mpm_runtime.hip", "mpm_server.hip",
           "mpm_noalloc.hip", "fem_kernels.hip", "fem_runtime.hip", "rb_kernels.hip", "rb_runtime.hip"]
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, extra=None, jobs: int = 0) -> str:
    """Compile every source to an object (in parallel), then link the shared library."""
    out_dir = os.path.join(HERE, "_build")
    os.makedirs(out_dir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(out_dir, src.replace(".hip", ".o"))
        cmds.append([hipcc()] + FLAGS + list(extra or []) + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for c, r in zip(cmds, ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds)):
            if r.returncode != 0:
                raise RuntimeError(f"hipcc failed ({r.returncode}): {' '.join(c)}\n{r.stdout}{r.stderr}")
            if verbose and r.stderr.strip():
                print("\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l), flush=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
