#!/usr/bin/env python3
"""Derive the polynomial and rational coefficients of the device special
functions and write them to mds_coeffs.h (a build input of the HIP library).

    python paper_1905_04582_amd/csrc/gen_coeffs.py

Everything is computed here from the mathematics with mpmath (50 digits):

* erfcx(z) = exp(z^2) erfc(z) on [0, Z] by one rational function P(z)/Q(z)
  (deg P = n-1, deg Q = n, Q(0) = 1), fitted by iteratively reweighted linear
  least squares (Loeb's linearisation with Lawson weights, which converges
  towards the minimax fit in relative error).  Z is where exp(-z^2) leaves the
  range of the format (FP64: z^2 > 745; FP32: z^2 > 104), beyond which the
  product exp(-z^2) erfcx(z) is 0 whatever erfcx is.  A second, shorter FP64
  rational covers [2.1, 6.6] only (t = z sqrt 2 from 2.97 to 9.33), for the
  wavefronts whose pairs all lie at t >= 3.
* exp(r) on |r| <= ln(2)/2 by its Taylor polynomial (FP64), after the
  Cody-Waite reduction x = k ln 2 + r with ln 2 split into a head with 20
  trailing zero bits and a tail.
* atanh(sqrt(v))/sqrt(v) = sum_k v^k/(2k+1) on 0 <= v <= 1/9 by Chebyshev
  interpolation (near-minimax), for log1p(-q) = -2 s A(s^2), s = q/(2-q),
  q in [0, 1/2].

Each fit is checked with its coefficients rounded to the target format and
evaluated by Horner's rule in that format; the measured worst relative
errors are written into the header.
"""
from __future__ import annotations

import os
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 50
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "mds_coeffs.h")


def erfcx(z):
    return mp.erfc(z) * mp.exp(z * z)


def fit_erfcx(n: int, zmax, npts: int = 500, iters: int = 12, zmin=0):
    zmin = mp.mpf(zmin)
    xs = [zmin + (zmax - zmin) * (mp.mpf(1) / 2 - mp.cos(mp.pi * (k + mp.mpf(1) / 2) / npts) / 2)
          for k in range(npts)]
    ys = [erfcx(x) for x in xs]
    w = [mp.mpf(1)] * npts
    qprev = [mp.mpf(1)] * npts
    best = None
    for _ in range(iters):
        A = mp.matrix(npts, 2 * n)
        b = mp.matrix(npts, 1)
        for i, (x, y) in enumerate(zip(xs, ys)):
            s = w[i] / (y * qprev[i])
            xp = mp.mpf(1)
            for k in range(n):          # p_0 .. p_{n-1}
                A[i, k] = s * xp
                xp *= x
            xp = x
            for k in range(n):          # q_1 .. q_n  (q_0 = 1)
                A[i, n + k] = -s * y * xp
                xp *= x
            b[i] = s * y
        sol = mp.qr_solve(A, b)[0]
        p = [sol[k] for k in range(n)]
        q = [mp.mpf(1)] + [sol[n + k] for k in range(n)]
        errs = [(mp.polyval(p[::-1], x) / mp.polyval(q[::-1], x) - y) / y for x, y in zip(xs, ys)]
        qprev = [mp.polyval(q[::-1], x) for x in xs]
        m = max(abs(e) for e in errs)
        if best is None or m < best[0]:
            best = (m, p, q)
        w = [w[i] * mp.sqrt(abs(errs[i])) for i in range(npts)]
        sw = sum(w)
        w = [wi / sw * npts for wi in w]
    return best[1], best[2]


def horner_np(c, x, dt):
    """Horner's rule in dtype dt (FMA emulated in float64/longdouble exactness
    is not needed for the error estimate: each step is rounded to dt)."""
    c = [dt(v) for v in c]
    acc = np.full_like(x, c[-1], dtype=dt)
    for v in c[-2::-1]:
        acc = (acc.astype(np.longdouble) * x.astype(np.longdouble) + np.longdouble(v)).astype(dt)
    return acc


def check_erfcx(p, q, zmax, dt, zmin=0.0):
    zs = np.linspace(float(zmin), float(zmax), 4001).astype(dt)
    P = horner_np([float(v) for v in p], zs, dt)
    Q = horner_np([float(v) for v in q], zs, dt)
    r = (P.astype(np.longdouble) / Q.astype(np.longdouble))
    ref = np.array([float(erfcx(mp.mpf(float(z)))) for z in zs], dtype=np.longdouble)
    return float(np.max(np.abs(r - ref) / ref))


def cheb_fit(f, a, b, deg):
    """Monomial coefficients (in v) of the Chebyshev interpolant of f on [a, b]."""
    nodes = [(a + b) / 2 + (b - a) / 2 * mp.cos(mp.pi * (k + mp.mpf(1) / 2) / (deg + 1))
             for k in range(deg + 1)]
    V = mp.matrix(deg + 1, deg + 1)
    rhs = mp.matrix(deg + 1, 1)
    for i, x in enumerate(nodes):
        for k in range(deg + 1):
            V[i, k] = x ** k
        rhs[i] = f(x)
    c = mp.lu_solve(V, rhs)
    return [c[k] for k in range(deg + 1)]


def atanh_ratio(v):
    if v == 0:
        return mp.mpf(1)
    s = mp.sqrt(v)
    return mp.atanh(s) / s


def check_poly(c, f, a, b, dt):
    xs = np.linspace(float(a), float(b), 4001).astype(dt)
    got = horner_np([float(v) for v in c], xs, dt).astype(np.longdouble)
    ref = np.array([float(f(mp.mpf(float(x)))) for x in xs], dtype=np.longdouble)
    return float(np.max(np.abs(got - ref) / np.abs(ref)))


def fmt(v, dt):
    if dt is np.float64:
        return float(v).hex()
    return float(np.float32(float(v))).hex() + "f"


def emit_array(name, vals, dt):
    # FP64 tables end up in constant memory (mds_math.h gathers them into one
    # object): VOP3 instructions on gfx950 take no 64-bit literal, but they do
    # take a scalar-register operand, so uniform loads of the table let every
    # Horner step be one v_fma_f64.  FP32 coefficients fit the 32-bit literal
    # field and stay compile-time constants.
    body = ",\n    ".join(fmt(v, dt) for v in vals)
    if dt is np.float64:
        return f"constexpr double {name}[{len(vals)}] = {{\n    {body}}};\n"
    return f"constexpr float {name}[{len(vals)}] = {{\n    {body}}};\n"


def main():
    lines = ["// mds_coeffs.h -- generated by gen_coeffs.py; do not edit by hand.",
             "// Coefficients are listed from the constant term upwards (Horner order reversed).",
             "#pragma once", "", "#include <hip/hip_runtime.h>", "", "namespace mds {", ""]

    # ---- erfcx rationals
    z64 = mp.mpf("27.5")     # exp(-z^2) underflows to 0 in FP64 beyond z^2 ~ 745
    z32 = mp.mpf("10.25")    # and in FP32 beyond z^2 ~ 104
    p64, q64 = fit_erfcx(10, z64)
    p32, q32 = fit_erfcx(5, z32)
    e64 = check_erfcx(p64, q64, z64, np.float64)
    e32 = check_erfcx(p32, q32, z32, np.float32)
    lines.append(f"// erfcx(z) ~ P(z)/Q(z) on [0, {z64}] (FP64); worst relative error "
                 f"{e64:.2e} with FP64 coefficients")
    lines.append(f"constexpr double kErfcxZmax64 = {float(z64)!r};")
    lines.append(emit_array("kErfcxP64", p64, np.float64))
    lines.append(emit_array("kErfcxQ64", q64, np.float64))
    lines.append(f"// erfcx(z) ~ P(z)/Q(z) on [0, {z32}] (FP32); worst relative error "
                 f"{e32:.2e} with FP32 coefficients")
    lines.append(f"constexpr float kErfcxZmax32 = {float(z32)!r}f;")
    lines.append(emit_array("kErfcxP32", p32, np.float32))
    lines.append(emit_array("kErfcxQ32", q32, np.float32))
    # the far range: every pair of the wavefront at t >= 3
    zf0, zf1, tfar = mp.mpf("2.1"), mp.mpf("6.6"), 3.0
    pf, qf = fit_erfcx(7, zf1, zmin=zf0)
    ef = check_erfcx(pf, qf, zf1, np.float64, zmin=zf0)
    lines.append(f"// erfcx(z) ~ P(z)/Q(z) on [{zf0}, {zf1}] (FP64, t = z sqrt 2 >= {tfar} up to "
                 f"rounding); worst relative error {ef:.2e} with FP64 coefficients")
    lines.append(f"constexpr double kFarT = {tfar!r};")
    lines.append(f"constexpr double kErfcxFarZmin64 = {float(zf0)!r};")
    lines.append(f"constexpr double kErfcxFarZmax64 = {float(zf1)!r};")
    lines.append(emit_array("kErfcxFarP64", pf, np.float64))
    lines.append(emit_array("kErfcxFarQ64", qf, np.float64))

    # ---- exp: Cody-Waite split of ln 2 and Taylor coefficients
    ln2 = mp.log(2)
    m, e = mp.frexp(ln2)
    head = mp.ldexp(mp.floor(mp.ldexp(m, 33)), e - 33)   # 33 significant bits
    tail = ln2 - head
    degx = 12
    taylor = [1 / mp.factorial(k) for k in range(degx + 1)]
    rmax = ln2 / 2
    ex_err = check_poly(taylor, mp.exp, -rmax, rmax, np.float64)
    lines.append("// exp(x) = 2^k exp(r), x = k ln2 + r, |r| <= ln2/2; ln2 = head + tail with")
    lines.append("// head on 33 significant bits so that k*head is exact for |k| < 2^20")
    lines.append(f"constexpr double kLn2Head = {float(head).hex()};")
    lines.append(f"constexpr double kLn2Tail = {float(tail).hex()};")
    lines.append(f"constexpr double kLog2e = {float(1 / ln2).hex()};")
    lines.append(f"// Taylor polynomial of exp(r), degree {degx}; worst relative error {ex_err:.2e}")
    lines.append(emit_array("kExpC64", taylor, np.float64))

    # ---- atanh series for log1p(-q)
    vmax = mp.mpf(1) / 9
    d64, d32 = 11, 5
    a64 = cheb_fit(atanh_ratio, mp.mpf(0), vmax, d64)
    a32 = cheb_fit(atanh_ratio, mp.mpf(0), vmax, d32)
    ea64 = check_poly(a64, atanh_ratio, 0, vmax, np.float64)
    ea32 = check_poly(a32, atanh_ratio, 0, vmax, np.float32)
    lines.append("// A(v) = atanh(sqrt v)/sqrt v on [0, 1/9], so that log1p(-q) = -2 s A(s^2),")
    lines.append(f"// s = q/(2-q); FP64 degree {d64}: worst relative error {ea64:.2e}; "
                 f"FP32 degree {d32}: {ea32:.2e}")
    lines.append(emit_array("kAtanhA64", a64, np.float64))
    lines.append(emit_array("kAtanhA32", a32, np.float32))

    lines += ["}  // namespace mds", ""]
    with open(OUT, "w") as f:
        f.write("\n".join(lines))
    print(f"wrote {OUT}: erfcx64 {e64:.2e} erfcx32 {e32:.2e} erfcx-far {ef:.2e} exp {ex_err:.2e} "
          f"atanh64 {ea64:.2e} atanh32 {ea32:.2e}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
