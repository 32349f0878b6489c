"""The quartet kernels read the Boys-function table row of a near lane without clamping its
index: a lane is near only for |P-Q|^2 < 32/rho, and T' = |P-Q|^2 rho/h is then below
32/h = 384 rows (FP64 grid, h = 1/12) or 512 (FP32 grid, h = 1/16) up to rounding, well
inside the 393 and 536 rows the tables hold.  These CPU checks take the largest |P-Q|^2 that
still passes the switch test in each precision, round T' as the kernels do (once, to the
nearest integer: the rounding constant 1.5 2^52 or 1.5 2^23 leaves an ulp of 1), and check
the row, for every exponent combination of the He and H contractions and for random ones."""
import os
import re
from fractions import Fraction

import numpy as np

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "paper_2509_21039_amd", "csrc", "hfk_internal.hpp")


def _constant(name):
    m = re.search(r"constexpr\s+(?:double|int)\s+%s\s*=\s*([0-9.]+)\s*;" % name, open(HEADER).read())
    assert m, name
    return float(m.group(1))


# the kernels' grid constants, read from their header
T_SWITCH = _constant("kTswitch")
GRIDS = {  # precision: (1/h, rows in the table)
    "fp64": (_constant("kBoysInvH"), int(_constant("kBoysGrid"))),
    "fp32": (_constant("kBoysInvHF"), int(_constant("kBoysGridF"))),
}
HE = (6.36242139, 1.158923, 0.31364979)
H = (3.42525091, 0.62391373, 0.16885540)


def _row(r2, rsh):
    """Round-half-even of the exact product, as the FMA with the rounding constant does."""
    t = Fraction(float(r2)) * Fraction(float(rsh))
    q, rem = divmod(t.numerator, t.denominator)
    twice = 2 * rem
    if twice > t.denominator or (twice == t.denominator and q % 2 == 1):
        q += 1
    return q


def _rhos(rng):
    alphas = list(HE) + list(H)
    ps = [a + b for a in alphas for b in alphas]
    out = [p * q / (p + q) for p in ps for q in ps]
    ps_r = np.exp(rng.uniform(np.log(0.05), np.log(200.0), size=(2000, 2)))
    out += list(ps_r[:, 0] * ps_r[:, 1] / (ps_r[:, 0] + ps_r[:, 1]))
    return out


def test_near_lane_rows_stay_inside_the_tables():
    rng = np.random.default_rng(11)
    for prec, (inv_h, rows) in GRIDS.items():
        top = int(T_SWITCH * inv_h)
        assert top < rows
        worst = 0
        for rho in _rhos(rng):
            if prec == "fp64":
                sw = np.float64(T_SWITCH / rho)
                rsh = np.float64(rho * inv_h)
                r2 = np.nextafter(sw, np.float64(0.0))        # the largest |P-Q|^2 below the switch
            else:
                sw = np.float32(T_SWITCH / rho)
                rsh = np.float32(rho * inv_h)
                r2 = np.nextafter(sw, np.float32(0.0))
            k = _row(r2, rsh)
            worst = max(worst, k)
            assert 0 <= k <= top, (prec, rho, k)
        assert worst == top   # the bound is reached, so the check is not vacuous


def test_per_atom_rows_keep_their_margin():
    """Per-atom bases derive rho/h from the switch radius^2 through a reciprocal square root
    (a Newton step in FP64, the hardware estimate in FP32): even a relative error of 1e-5 in
    rho/h, far above either, keeps T' below top + 1/2."""
    for inv_h, _ in GRIDS.values():
        top = T_SWITCH * inv_h
        assert top * (1.0 + 1e-5) < top + 0.5


def test_rounding_rule_matches_half_even():
    assert _row(1.5, 1.0) == 2 and _row(2.5, 1.0) == 2 and _row(0.49, 1.0) == 0
    assert _row(383.5, 1.0) == 384 and _row(384.4999, 1.0) == 384
