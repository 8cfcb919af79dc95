"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU:

- the oracle: every oracle pin and analysis test, run in a child process
  against a sanitized build of gbr_oracle.c;
- the C ABI's host side: the library built with the sanitizers on its host
  code (device code compiled as usual, nothing launched), driven by a small C
  program through every argument check that runs before a device is touched,
  including offsets whose differences overflow 32 bits;
- the work-list builders of pair_list.h are exercised sanitized by the
  harnesses of test_pair_list_cpu.py, which build with the same flags.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1809_07726_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}

DRIVER = r"""
#include <limits.h>
#include <stdio.h>
#include <stdlib.h>
#include "gbremd.h"

static int fails = 0;
#define EXPECT(call, code) do { int rc_ = (call); if (rc_ != (code)) { \
    printf("FAIL %s: %d != %d (%s)\n", #call, rc_, code, gbr_last_error()); ++fails; } } while (0)

int main(void) {
    gbr_gb_params p = {332.0522173, 1.0, 78.5, 0.09, 1.0, 0.8, 4.85, 0.0, 0.0, 0.0};
    gbr_ctx* h = 0;
    int32_t off[3] = {0, 5, 9};
    EXPECT(gbr_ctx_create(0, &p, 2, off), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, 0, 2, off), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, 0, off), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, -5, off), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, 1 << 30, off), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, 2, 0), GBR_E_INVAL);
    int32_t empty[3] = {0, 5, 5}, first[3] = {1, 5, 9}, down[3] = {0, 9, 5};
    EXPECT(gbr_ctx_create(&h, &p, 2, empty), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, 2, first), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, 2, down), GBR_E_INVAL);
    int32_t wide[3] = {0, 5, INT_MIN}, wide2[3] = {0, INT_MAX, INT_MIN};
    EXPECT(gbr_ctx_create(&h, &p, 2, wide), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, 2, wide2), GBR_E_INVAL);
    int32_t big[2] = {0, INT_MAX};
    EXPECT(gbr_ctx_create(&h, &p, 1, big), GBR_E_INVAL);
    enum { NB = 257 };                         /* 257 replicas of 2^20 atoms: over GBR_MAX_ATOMS */
    int32_t* many = (int32_t*)malloc(sizeof(int32_t) * (NB + 1));
    for (int r = 0; r <= NB; ++r) many[r] = r << 20;
    EXPECT(gbr_ctx_create(&h, &p, NB, many), GBR_E_INVAL);
    free(many);
    gbr_gb_params q = p; q.eps_out = -1.0;
    EXPECT(gbr_ctx_create(&h, &q, 2, off), GBR_E_INVAL);
    q = p; q.kappa = 1.0 / 0.0;
    EXPECT(gbr_ctx_create(&h, &q, 2, off), GBR_E_INVAL);
    q = p; q.cut = 0.0 / 0.0;
    EXPECT(gbr_ctx_create(&h, &q, 2, off), GBR_E_INVAL);
    EXPECT(gbr_ctx_create(&h, &p, 2, off), GBR_E_NODEVICE);      /* a valid layout, no device */
    if (h) { printf("FAIL: a context without a device\n"); ++fails; }

    EXPECT(gbr_ctx_destroy(0), GBR_OK);
    EXPECT(gbr_check(0, 0, 0), GBR_E_INVAL);
    EXPECT(gbr_ctx_sizes(0, 0, 0, 0), GBR_E_INVAL);
    EXPECT(gbr_set_launch(0, 4, 8), GBR_E_INVAL);
    EXPECT(gbr_set_blocking(0, 1, 1, 1), GBR_E_INVAL);
    EXPECT(gbr_set_split(0, 16), GBR_E_INVAL);
    EXPECT(gbr_set_timing(0, 1), GBR_E_INVAL);
    EXPECT(gbr_get_timing(0, 0, 0), GBR_E_INVAL);
    EXPECT(gb_born_radii(0, 0, 0, 0, 0, 0, 0, 0), GBR_E_INVAL);
    EXPECT(gb_energy_forces(0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0), GBR_E_INVAL);
    EXPECT(titration_delta_e(0, 0, 0, 0, 0, 0, 0, 0, 0), GBR_E_INVAL);
    EXPECT(remd_exchange(0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0), GBR_E_INVAL);
    EXPECT(md_step(0, 0, 0, 0, 0, 1, 0, 0), GBR_E_INVAL);
    EXPECT(gbr_fx_to_float(0, 0, 0, 0, 0, 0, 0, 0), GBR_E_INVAL);
    EXPECT(gbr_energies(0, 0, 0, 0), GBR_E_INVAL);
    EXPECT(gbr_exchange_inputs(0, 0, 0, 0, 0, 0, 0, 0), GBR_E_INVAL);

    float f[4] = {0};
    double d[4] = {0};
    uint32_t e = 0;
    EXPECT(gb_born_radii_noalloc(0, 1, off, 9, 9, f, f, f, f, f, d, &e, 0), GBR_E_INVAL);
    EXPECT(gb_born_radii_noalloc(&p, 0, off, 9, 9, f, f, f, f, f, d, &e, 0), GBR_E_INVAL);
    EXPECT(gb_born_radii_noalloc(&p, 2, off, 0, 1, f, f, f, f, f, d, &e, 0), GBR_E_INVAL);
    EXPECT(gb_born_radii_noalloc(&p, 2, off, GBR_NOALLOC_MAX_ATOMS + 1, 9, f, f, f, f, f, d, &e, 0),
           GBR_E_INVAL);
    EXPECT(gb_born_radii_noalloc(&p, 2, off, 9, 10, f, f, f, f, f, d, &e, 0), GBR_E_INVAL);
    EXPECT(gb_born_radii_noalloc(&p, 1 << 25, off, GBR_NOALLOC_MAX_ATOMS, GBR_NOALLOC_MAX_ATOMS,
                                 f, f, f, f, f, d, &e, 0), GBR_E_INVAL);
    q = p; q.rgbmax = -1.0;
    EXPECT(gb_born_radii_noalloc(&q, 2, off, 9, 5, f, f, f, f, f, d, &e, 0), GBR_E_INVAL);
    printf("%s: %d failures\n", fails ? "FAILED" : "OK", fails);
    return fails != 0;
}
"""


def _env(**extra):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(extra)
    return env


def test_capi_host_checks_under_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc not available")
    from paper_1809_07726_amd.build import FLAGS, SOURCES
    flags = [f for f in FLAGS if f != "-O3"]
    host_san = [x for s in SAN for x in ("-Xarch_host", s)]
    objs = []
    procs = []
    for src in SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, "-O1", *host_san, "-c", os.path.join(CSRC, src), "-o", obj],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err
    drv_c, drv_o, exe = tmp_path / "drv.c", str(tmp_path / "drv.o"), str(tmp_path / "drv")
    drv_c.write_text(DRIVER)
    subprocess.check_call([CLANG, *SAN, "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-I", INCLUDE,
                           "-c", str(drv_c), "-o", drv_o])
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-fsanitize=address,undefined", drv_o, *objs,
                           "-o", exe])
    r = subprocess.run([exe], env=_env(HIP_VISIBLE_DEVICES=""), capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "OK: 0 failures" in r.stdout, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


def test_oracle_pins_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["gcc", *SAN, "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", lib,
                           os.path.join(ROOT, "oracle", "gbr_oracle.c"), "-lm"])
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    env = _env(GBR_ORACLE_LIB=lib, LD_PRELOAD=asan)
    check = "import oracle; oracle.lib(); print(any('liboracle_san' in l for l in open('/proc/self/maps')))"
    assert subprocess.check_output([sys.executable, "-c", check], env=env, cwd=ROOT, text=True).strip() == "True"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_pins.py", "tests/test_analysis_cpu.py"],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
