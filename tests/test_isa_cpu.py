"""Device code of the library and of the issue-rate microbenchmark compiled
to gfx950 assembly (hipcc -S, no GPU needed): no scalar-memory writes of any
kind, no packed FP32 arithmetic (the build disables it), no register spills
in the force-only pair kernels, and no FP64 arithmetic in the pair kernels."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_07726_amd", "csrc")
SOURCES = ["pair_kernels.hip", "atom_kernels.hip", "md_kernels.hip", "capi.hip", "../microbench/issue_rate.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SCALAR_WRITE = re.compile(r"^\s+s_(store|buffer_store|atomic|buffer_atomic|scratch_store|dcache_wb|dcache_discard)\w*\b",
                          re.M)
PACKED_F32 = re.compile(r"^\s+v_pk_(add|mul|fma|mov)_f32\b", re.M)


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_1809_07726_amd.build import FLAGS
    d = tmp_path_factory.mktemp("isa")
    out = {}
    for src in SOURCES:
        dst = d / (os.path.basename(src) + ".s")
        subprocess.check_call([HIPCC, *FLAGS, "--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", str(dst)],
                              stderr=subprocess.DEVNULL)
        out[src] = dst.read_text()
    return out


@pytest.mark.parametrize("src", SOURCES)
def test_no_scalar_memory_writes(asm, src):
    assert not SCALAR_WRITE.findall(asm[src])


@pytest.mark.parametrize("src", SOURCES)
def test_no_packed_fp32(asm, src):
    assert not PACKED_F32.findall(asm[src])


def test_force_only_pair_kernels_do_not_spill(asm):
    text = asm["pair_kernels.hip"]
    kernels = re.findall(r"^(_Z\S+):.*?; ScratchSize: (\d+)", text, re.M | re.S)
    assert kernels
    for name, scratch in kernels:
        grad = "ELb1E" in name                  # dE/dq or dE/drho variants
        if not grad:
            assert int(scratch) == 0, name


def test_pair_kernels_hold_no_fp64_arithmetic(asm):
    """The pair passes are FP32 throughout: partials reach fixed point through
    FP32 instructions and energies are summed over the wavefront as integers."""
    assert not re.findall(r"^\s+v_\w+_f64\b", asm["pair_kernels.hip"], re.M)
