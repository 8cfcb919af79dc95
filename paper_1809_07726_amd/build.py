"""Builds libgbremd.so (all HIP sources, gfx950) in the package directory, and
the issue-rate microbenchmark's libissue_rate.so next to its source.

Usage: python -m paper_1809_07726_amd.build   (or build() from Python)."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgbremd.so")
SOURCES = ["pair_kernels.hip", "atom_kernels.hip", "md_kernels.hip", "capi.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC]


def _compile(src, obj):
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature: drop that one warning
    return "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())


def build(verbose: bool = True) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_hct_poly.py")],
                          stdout=subprocess.DEVNULL)
    objs = [os.path.join(objdir, s.replace(".hip", ".o")) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        for src, msg in zip(SOURCES, ex.map(_compile, SOURCES, objs)):
            if msg and verbose:
                print(f"[{src}] {msg}")
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    from paper_1809_07726_amd.microbench import issue_rate   # the VALU issue-rate microbenchmark
    issue_rate.build()
    return LIB


if __name__ == "__main__":
    print(build())
