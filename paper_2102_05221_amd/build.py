"""Build libeap.so (HIP, gfx950) in-tree.

Every source under csrc/ is compiled by hipcc for gfx950 only, with FMA
contraction off (the cell formulas have a fixed operation order) and packed
FP32 instructions disabled, then linked into paper_2102_05221_amd/libeap.so.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

try:
    from . import srchash
except ImportError:   # run as a script
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2102_05221_amd import srchash

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libeap.so")
ARCH = os.environ.get("EAP_OFFLOAD_ARCH", "gfx950")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]

SOURCES = ["eap_rows.hip", "eap_band.hip", "eap_aux.hip", "eap_api.cpp", "eap_serve.cpp"]
# The sweep kernels are built with -fno-honor-nans: none of their cells is ever
# NaN, so min/max need no quieting of signalling NaNs and values are unchanged
# (no reassociation or contraction).  The host-side ABI is not: its argument
# checks must see NaN.
NO_NANS = {"eap_rows.hip", "eap_band.hip"}


def _compile(src: str, verbose: bool, digest: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    extra = ["-fno-honor-nans"] if src in NO_NANS else []
    if src == "eap_api.cpp":   # eap_source_hash(): the sources this library was built from
        extra.append(f'-DEAP_SOURCE_HASH="{digest}"')
    cmd = ["hipcc", *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    digest = srchash.source_hash()
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, digest), SOURCES))
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
