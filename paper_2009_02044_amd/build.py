"""Compile the HIP library libglasma.so for gfx950 in-tree (hipcc, no JIT cache)."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libglasma.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["capi.hip", "step.hip", "observe.hip", "init.hip", "semi.hip", "semi_march.hip", "adjoint.hip",
           "bi.hip"]

FLAGS = [
    "-O3", "-std=c++20", "-fPIC", "--offload-arch=gfx950",
    # packed FP32 instructions stay off: plain scalar FP32 arithmetic only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wno-unused-result",
]


def _compile(src, objdir, extra):
    obj = os.path.join(objdir, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


PROBES = ["valu_probe", "hbm_probe"]


def build_probe(verbose=False):
    """The stand-alone probes (executables, not part of the library): the VALU issue rate per
    instruction form and the achievable memory bandwidth."""
    outs = []
    for name in PROBES:
        out = os.path.join(HERE, name)
        tmp = out + ".tmp"
        r = subprocess.run(["hipcc", *[f for f in FLAGS if f != "-fPIC"], os.path.join(CSRC, name + ".hip"), "-o",
                            tmp], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {name}.hip:\n{r.stderr}")
        os.replace(tmp, out)
        if verbose:
            print("built", out)
        outs.append(out)
    return outs


def build(verbose=False, extra_flags=(), out=None):
    """Compile every source and link the shared library (out: path of the .so)."""
    out = out or OUT
    objdir = OBJ if out == OUT else out + ".objs"
    os.makedirs(objdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, objdir, list(extra_flags)), SOURCES))
    tmp = out + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    build_probe(verbose=True)
    sys.exit(0)
