"""The device special functions' coefficient tables (csrc/mds_coeffs.h)
against mpmath: each fitted rational or polynomial, evaluated by Horner's
rule in the table's own precision at points spread over its range, stays
within a few units in the last place of the function it stands for.  The
tables are read from the header as written (hex floats), so a stale or
hand-edited header fails here whatever the generator would produce."""
import os
import re

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1905_04582_amd", "csrc", "mds_coeffs.h")
mp.mp.dps = 40


def _tables():
    src = open(HEADER).read()
    arrays = {}
    for m in re.finditer(r"constexpr (double|float) (\w+)\[\d+\] = \{([^}]*)\};", src):
        vals = [v.strip().rstrip("f") for v in m.group(3).split(",") if v.strip()]
        arrays[m.group(2)] = [float.fromhex(v) for v in vals]
    scalars = {}
    for m in re.finditer(r"constexpr (double|float) (\w+) = ([^;\[]+);", src):
        v = m.group(3).strip().rstrip("f")
        scalars[m.group(2)] = float.fromhex(v) if "0x" in v else float(v)
    return arrays, scalars


ARR, SCAL = _tables()


def _horner(c, x, dt):
    acc = np.full_like(x, dt(c[-1]), dtype=dt)
    for v in c[-2::-1]:
        acc = (acc.astype(np.longdouble) * x.astype(np.longdouble) + np.longdouble(dt(v))).astype(dt)
    return acc


def _erfcx(z):
    return mp.erfc(z) * mp.exp(z * z)


def _max_rel(got, f, xs):
    ref = np.array([float(f(mp.mpf(float(x)))) for x in xs], dtype=np.longdouble)
    return float(np.max(np.abs(got.astype(np.longdouble) - ref) / np.abs(ref)))


@pytest.mark.parametrize("p,q,lo,hi,dt,tol", [
    ("kErfcxP64", "kErfcxQ64", 0.0, "kErfcxZmax64", np.float64, 2e-15),
    ("kErfcxFarP64", "kErfcxFarQ64", "kErfcxFarZmin64", "kErfcxFarZmax64", np.float64, 2e-15),
    ("kErfcxP32", "kErfcxQ32", 0.0, "kErfcxZmax32", np.float32, 1e-6),
])
def test_erfcx_rationals(p, q, lo, hi, dt, tol):
    lo = SCAL[lo] if isinstance(lo, str) else lo
    hi = SCAL[hi]
    zs = np.linspace(lo, hi, 701).astype(dt)
    got = (_horner(ARR[p], zs, dt).astype(np.longdouble) /
           _horner(ARR[q], zs, dt).astype(np.longdouble))
    assert ARR[q][0] == 1.0
    assert _max_rel(got, _erfcx, zs) < tol


def test_far_range_covers_the_far_steps():
    # t >= kFarT (less a few ulp of the squared-distance test) maps into the
    # far fit's range; the top of the range is where exp(-t^2/2) < 1e-18
    assert SCAL["kErfcxFarZmin64"] * np.sqrt(2.0) < SCAL["kFarT"] * (1 - 1e-12)
    assert np.exp(-(SCAL["kErfcxFarZmax64"] * np.sqrt(2.0)) ** 2 / 2) < 1e-18


def test_exp_taylor_and_cody_waite_split():
    ln2 = mp.log(2)
    # head + tail carries ln 2 to the precision of a double below 2^-34
    assert abs(mp.mpf(SCAL["kLn2Head"]) + mp.mpf(SCAL["kLn2Tail"]) - ln2) < mp.mpf(2) ** -85
    # the head's low bits are zero, so k * head is exact for |k| < 2^20
    m, e = np.frexp(SCAL["kLn2Head"])
    assert float(m * 2.0 ** 33) == np.floor(m * 2.0 ** 33)
    r = np.linspace(-float(ln2) / 2, float(ln2) / 2, 701)
    assert _max_rel(_horner(ARR["kExpC64"], r, np.float64), mp.exp, r) < 1e-15


@pytest.mark.parametrize("name,dt,tol", [("kAtanhA64", np.float64, 1e-15),
                                         ("kAtanhA32", np.float32, 3e-7)])
def test_atanh_ratio(name, dt, tol):
    def f(v):
        return mp.mpf(1) if v == 0 else mp.atanh(mp.sqrt(v)) / mp.sqrt(v)
    v = np.linspace(0.0, 1.0 / 9.0, 401).astype(dt)
    assert _max_rel(_horner(ARR[name], v, dt), f, v) < tol
