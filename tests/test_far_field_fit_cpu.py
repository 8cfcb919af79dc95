"""The far-sphere descreening fits used by the pair kernels (hct_poly.h, written
by csrc/gen_hct_poly.py) against the oracle's FP64 closed form of the HCT term
and its radial derivative (Theory, the OBC Born radii): for a sphere whose near
edge lies outside the atom, h = (x^3/r) G(x^2) and dh/dr = -(x^3/r^2) Q(x^2)
with x = s/r, on the whole fitted range x <= XMAX."""
import os
import re

import numpy as np
import pytest

import oracle

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_1809_07726_amd", "csrc", "hct_poly.h")


def _header():
    text = open(HDR).read()
    xmax = float(re.search(r"#define HCT_FAR_XMAX ([0-9.eE+-]+)f", text).group(1))
    coef = {}
    for name in ("G", "Q"):
        body = re.search(r"hct_%s_coef\[[^]]*\] = \{([^}]*)\}" % name, text).group(1)
        coef[name] = np.array([float(v.strip().rstrip("f")) for v in body.split(",")])
    return xmax, coef


def _horner(c, y):
    p = np.zeros_like(y) + c[-1]
    for k in range(len(c) - 2, -1, -1):
        p = p * y + c[k]
    return p


@pytest.mark.parametrize("r", [4.0, 9.0, 25.0])
def test_fits_match_closed_form(r):
    xmax, coef = _header()
    assert 0.3 <= xmax <= 0.5
    rt = 0.5 * r * (1.0 - xmax)                  # near edge r - s >= rt for every x <= xmax
    xs = np.linspace(0.05, xmax, 60)
    worst_h = worst_d = 0.0
    for x in xs:
        s = x * r
        assert r - s >= rt
        h = oracle.hct(r, rt, s)
        dh = oracle.hct_grad(r, rt, s)[0]
        h_fit = x ** 3 / r * _horner(coef["G"], np.array(x * x))
        d_fit = -x ** 3 / r ** 2 * _horner(coef["Q"], np.array(x * x))
        worst_h = max(worst_h, abs(h_fit / h - 1))
        worst_d = max(worst_d, abs(d_fit / dh - 1))
    # FP32 rounding is 6e-8; the fits stay within a few units of it
    assert worst_h < 1e-7, worst_h
    assert worst_d < 3e-7, worst_d
