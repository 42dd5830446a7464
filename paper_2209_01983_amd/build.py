"""Build libsale.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

    python -m paper_2209_01983_amd.build

The library lands next to this file, where the ctypes binding loads it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsale.so")
SOURCES = ["sale_step.hip", "sale_remap2.hip", "sale_lagrange.hip", "sale_pool.hip", "sale_noalloc.hip",
           "sale_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # FMA contraction (no fast-math): parity with the oracle stays at rounding level
    "-ffp-contract=fast",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-I", os.path.join(ROOT, "include"),
]


def build_lib(verbose: bool = False, extra=(), out: str = LIB) -> str:
    """Compile every source into libsale.so (always rebuilds). `extra`: more
    hipcc flags (e.g. -DSALE_WAVES_POOL=4 for a variant build); `out`: where
    the library goes (a variant is loaded by naming it in SALE_LIB)."""
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 feature and says so: harmless
    errs = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{r.stderr}")
    if verbose and errs:
        print(errs, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    import argparse

    ap = argparse.ArgumentParser(description="build libsale.so for gfx950")
    ap.add_argument("-D", dest="defines", action="append", default=[], metavar="NAME=VALUE",
                    help="a preprocessor definition of a variant build (repeatable)")
    ap.add_argument("--out", default=LIB, help="output path (default: next to the binding)")
    a = ap.parse_args()
    print(build_lib(verbose=True, extra=[f"-D{d}" for d in a.defines], out=os.path.abspath(a.out)))
