"""Build the HIP library (gfx950) in-tree: paper_2603_17711_amd/libtenso.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "checks.hip", "svd.hip", "vmf.hip", "tenso_host.cpp", "mlp.hip", "noalloc.hip")]
OUT = os.path.join(HERE, "libtenso.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(HERE, "..", "include")]


def _torch_libdir():
    import importlib.util
    spec = importlib.util.find_spec("torch")
    return os.path.join(os.path.dirname(spec.origin), "lib") if spec else None


def build(verbose=False):
    tmp = OUT + ".tmp"
    link = []
    tl = _torch_libdir()
    if tl:  # bind to the HIP runtime that torch ships (one runtime per process)
        link = ["-Wl,-rpath," + tl, "-Wl,--disable-new-dtags"]
    cmd = [HIPCC] + FLAGS + ["-x", "hip"] + SRC + ["-o", tmp] + link
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
