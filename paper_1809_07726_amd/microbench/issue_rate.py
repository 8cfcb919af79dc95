"""VALU issue-rate microbenchmark (gfx950): runs each instruction mix of
issue_rate.hip at 1, 2, 4 and 8 wavefronts per SIMD and prints a markdown
table of wave64 instructions issued per quad-cycle per SIMD over the kernel's
event-timed duration (2 = two VALU instructions issued together every
quad-cycle, the dual-issue limit; LDS instructions count as instructions).

Usage: python -m paper_1809_07726_amd.microbench.issue_rate [iters]
(builds libissue_rate.so next to this file when it is missing)."""
import ctypes as C
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "issue_rate.hip")
LIB = os.path.join(HERE, "libissue_rate.so")
MIXES = ("v_fmac_f32 (VOP2)", "v_fma_f32, negated operand (VOP3)", "v_mul_f32, SGPR operand",
         "v_fmaak_f32 (literal)", "v_exp_f32", "v_rsq_f32", "v_add_f32_dpp wave_rol:1",
         "12 v_fmac + 4 v_exp", "14 v_fmac + 2 v_exp", "12 v_fmac + 4 dpp", "8 v_fmac + 8 VOP3 v_fma",
         "8 v_fmac + 8 v_mul SGPR", "12 v_fmac + 4 ds_add_f32", "14 v_fmac + 2 ds_read_b128, each waited for",
         "12 v_fmac + 4 dpp row_ror:1", "12 v_fmac + 4 ds_bpermute_b32")


def build() -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", tmp],
                          stderr=subprocess.DEVNULL)
    os.replace(tmp, LIB)
    return LIB


def main(iters=20000):
    if not os.path.exists(LIB):
        build()
    L = C.CDLL(LIB)
    L.issue_rate_run.argtypes = [C.c_int, C.c_int, C.c_int] + [C.POINTER(C.c_double)] * 3
    W = (1, 2, 4, 8)
    print("| instruction mix | " + " | ".join(f"{w} wave/SIMD" for w in W) + " | clock MHz |")
    print("|---|" + "---|" * (len(W) + 1))
    for m in range(L.issue_rate_mix_count()):
        cells, mhz = [], 0.0
        for w in W:
            ipq, f, ms = C.c_double(), C.c_double(), C.c_double()
            rc = L.issue_rate_run(m, w, iters, C.byref(ipq), C.byref(f), C.byref(ms))
            if rc != 0:
                raise RuntimeError(f"issue_rate_run({m}, {w}) failed: {rc}")
            cells.append(f"{ipq.value:.2f}")
            mhz = max(mhz, f.value)
        print(f"| {MIXES[m]} | " + " | ".join(cells) + f" | {mhz:.0f} |", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 20000)
