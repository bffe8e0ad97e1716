"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from
mpmath brute force, scipy special functions, closed forms, invariants or
quadrature (Eq. 2 and Eq. 9 of the paper, Section 2.3 for the leapfrog).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate, special

import oracle
from tests import mp_reference as mpr

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_cases.json")


def _case(name):
    with open(GOLDEN) as f:
        c = json.load(f)["cases"][name]
    x = np.array(c["x"], dtype=np.float64)
    y = np.array(c["y"], dtype=np.float64)
    n = x.shape[0]
    mask = None
    if c["missing"]:
        mask = np.zeros((n, n), np.uint8)
        for i, j in c["missing"]:
            mask[i, j] = mask[j, i] = 1
    return x, y, mask, c["sigma"]


def _rel(a, b, scale=None):
    scale = abs(b) if scale is None else scale
    return abs(a - b) / max(scale, 1e-300)


# ------------------------------------------------------------- ln Phi -----

@pytest.mark.parametrize("t", [0.0, 1e-8, 0.3, 1.0, 2.5, 5.0, 8.0, 10.0, 20.0, 38.0,
                               -0.5, -3.0, -5.0, -5.0001, -7.5, -10.0, -25.0, -40.0])
def test_log_phi_vs_mpmath(t):
    ref = float(mpr.log_phi(t))
    got = float(oracle.log_phi(t))
    if ref == 0.0:
        assert got == 0.0
    else:
        # the t >= 0 branch must keep relative accuracy as Phi -> 1
        # (a naive log(Phi) loses all digits beyond t ~ 8.3); rounding t/sqrt(2)
        # alone perturbs Phi(-t) by ~t^2 ulp, hence the t-dependent bound
        assert _rel(got, ref) < 1e-15 * (5 + t * t), (t, got, ref)


def test_log_phi_special_values():
    assert float(oracle.log_phi(0.0)) == pytest.approx(-math.log(2.0), rel=1e-16, abs=0)
    # Phi is a CDF: ln Phi < 0 and increasing
    t = np.linspace(-40, 40, 4001)
    v = oracle.log_phi(t)
    assert np.all(v <= 0) and np.all(np.diff(v) >= 0)


def test_log_phi_vs_scipy_log_ndtr():
    t = np.concatenate([np.linspace(-40, 40, 2001), np.geomspace(1e-6, 37, 200)])
    ref = special.log_ndtr(t)
    got = oracle.log_phi(t)
    nz = ref != 0
    # both sides lose ~t^2 ulp to the rounding of the erfc argument
    bound = 2e-15 * (5 + t[nz] ** 2)
    assert np.all(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz]) < bound)


@pytest.mark.parametrize("t", [0.0, 0.5, 1.0, 3.0, 8.0, 20.0, -1.0, -3.0, -6.0, -10.0, -40.0])
def test_mills_vs_mpmath(t):
    ref = float(mpr.mills(t))
    got = float(oracle.mills(t))
    assert _rel(got, ref) < 1e-15 * (5 + t * t), (t, got, ref)


def test_mills_maximum_at_zero_on_halfline():
    # phi/Phi is decreasing on t >= 0, its value at 0 is sqrt(2/pi)
    assert float(oracle.mills(0.0)) == pytest.approx(math.sqrt(2 / math.pi), rel=1e-15)
    v = oracle.mills(np.linspace(0, 30, 3001))
    assert np.all(np.diff(v) <= 0)


# ------------------------------------------------------- tiny worked cases --

@pytest.mark.parametrize("name", ["C_two_points", "A_345_exact", "B_345_perturbed",
                                  "E_d3_one_missing"])
def test_tiny_cases_vs_brute_force(name):
    x, y, mask, sigma = _case(name)
    ref = mpr.brute_force(x, y, sigma, mask)
    ev = oracle.evaluate(x, y, sigma, mask)
    assert ev.m_obs == ref["m_obs"]
    assert _rel(ev.loglik, float(ref["loglik"])) < 1e-14
    assert _rel(ev.dsigma, float(ref["dsigma"])) < 1e-14
    gref = np.array([[float(v) for v in row] for row in ref["grad"]])
    scale = np.max(np.abs(gref))
    assert np.max(np.abs(ev.grad - gref)) <= 1e-14 * scale
    _check_scales(ev, ref)


def _check_scales(ev, ref, tol=1e-14):
    """The oracle's rounding scales -- A_i, B_i and the absolute sums of L and
    dL/dsigma, which set the tolerance of every GPU parity check -- against
    the same sums in mpmath."""
    for got, want in ((ev.absrow, ref["absrow"]), (ev.condrow, ref["condrow"])):
        want = np.array([float(v) for v in want])
        assert np.all(np.abs(got - want) <= tol * np.maximum(want, 1e-300)), (got, want)
    assert _rel(ev.abs_loglik, float(ref["abs_loglik"])) < tol
    assert _rel(ev.abs_dsigma, float(ref["abs_dsigma"])) < tol


def test_case_c_closed_form():
    # delta = 1, y = 2, sigma = 1 (one pair): L = -1/2 - ln Phi(1),
    # g_0 = (phi(1)/Phi(1) - 1, 0), dL/dsigma = -1 + 1 + phi(1)/Phi(1)
    x, y, mask, sigma = _case("C_two_points")
    ev = oracle.evaluate(x, y, sigma, mask)
    m1 = math.exp(-0.5) / math.sqrt(2 * math.pi) / special.ndtr(1.0)
    assert ev.loglik == pytest.approx(-0.5 - special.log_ndtr(1.0), rel=1e-15)
    assert ev.grad[0, 0] == pytest.approx(m1 - 1.0, rel=1e-14)
    assert ev.grad[1, 0] == pytest.approx(1.0 - m1, rel=1e-14)
    assert ev.grad[0, 1] == 0.0 and ev.grad[1, 1] == 0.0
    assert ev.dsigma == pytest.approx(m1, rel=1e-14)


def test_case_a_quadratic_term_vanishes():
    # y = delta: L = -sum ln Phi(delta/sigma) with sigma = 1
    x, y, mask, sigma = _case("A_345_exact")
    ev = oracle.evaluate(x, y, sigma, mask)
    ref = -(special.log_ndtr(3.0) + special.log_ndtr(4.0) + special.log_ndtr(5.0))
    assert ev.loglik == pytest.approx(ref, rel=1e-13)


# --------------------------------------------------- random brute force -----

def _rand_problem(n, d, sigma, seed, missing=0.0, nan_frac=0.0):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, d)) * 1.5
    y = np.abs(rng.standard_normal((n, n))) * 2 + 0.05
    y = np.tril(y, -1)
    y = y + y.T
    mask = None
    if missing > 0:
        m = np.tril(rng.random((n, n)) < missing, -1)
        mask = (m | m.T).astype(np.uint8)
    if nan_frac > 0:
        m = np.tril(rng.random((n, n)) < nan_frac, -1)
        y[m | m.T] = np.nan
    return x, y, mask


@pytest.mark.parametrize("n,d,sigma,seed,missing,nan_frac", [
    (2, 1, 0.7, 1, 0.0, 0.0), (5, 2, 0.3, 2, 0.0, 0.0), (6, 3, 1.7, 3, 0.3, 0.0),
    (7, 4, 0.9, 4, 0.0, 0.2), (8, 2, 0.05, 5, 0.2, 0.1), (6, 6, 2.5, 6, 0.0, 0.0)])
def test_random_vs_brute_force(n, d, sigma, seed, missing, nan_frac):
    x, y, mask = _rand_problem(n, d, sigma, seed, missing, nan_frac)
    ref = mpr.brute_force(x, y, sigma, mask)
    ev = oracle.evaluate(x, y, sigma, mask)
    assert ev.m_obs == ref["m_obs"] == oracle.count_observed(y, mask)
    assert _rel(ev.loglik, float(ref["loglik"]), ev.abs_loglik) < 1e-14
    assert _rel(ev.dsigma, float(ref["dsigma"]), ev.abs_dsigma) < 1e-14
    gref = np.array([[float(v) for v in row] for row in ref["grad"]])
    for i in range(n):
        assert np.max(np.abs(ev.grad[i] - gref[i])) <= 1e-14 * max(ev.absrow[i], 1e-300)
    _check_scales(ev, ref)


@pytest.mark.parametrize("seed", [31, 32])
def test_scales_of_untruncated_model_vs_brute_force(seed):
    # the untruncated evaluation's scales (the tolerances of its GPU checks)
    x, y, mask = _rand_problem(7, 3, 0.7, seed, missing=0.2, nan_frac=0.1)
    ref = mpr.brute_force(x, y, 0.7, mask, truncated=False)
    ev = oracle.evaluate(x, y, 0.7, mask, truncated=False)
    _check_scales(ev, ref)


def test_scale_of_a_pair_by_hand():
    # two points, delta = 1, y = 2, sigma = 0.5: w = (1 - 2)/0.25 + 2 m(2),
    # r = 1/(2 0.25) + ln Phi(2), ds = 1/0.125 + 4 m(2), with m(2) = phi(2)/Phi(2)
    x = np.array([[0.0], [1.0]])
    y = np.array([[0.0, 2.0], [2.0, 0.0]])
    ev = oracle.evaluate(x, y, 0.5)
    m2 = math.exp(-2.0) / math.sqrt(2 * math.pi) / special.ndtr(2.0)
    b = (1.0 + 2.0) / 0.25 + m2 / 0.5
    assert ev.condrow == pytest.approx([b, b], rel=1e-15)
    assert ev.absrow == pytest.approx([abs(-4.0 + 2 * m2)] * 2, rel=1e-15)
    assert ev.abs_loglik == pytest.approx(abs(2.0 + special.log_ndtr(2.0)) + math.log(2.0),
                                          rel=1e-15)
    assert ev.abs_dsigma == pytest.approx(8.0 + 4.0 * m2 + 2.0, rel=1e-15)


def test_coincident_points():
    # delta = 0: ln Phi(0) = -ln 2 enters L, the gradient term is zero
    x = np.array([[1.0, 2.0], [1.0, 2.0]])
    y = np.array([[0, 0.4], [0.4, 0]])
    ev = oracle.evaluate(x, y, 0.5)
    assert ev.loglik == pytest.approx(-math.log(0.5) - (0.4 ** 2 / 0.5 - math.log(2)), rel=1e-15)
    assert np.all(ev.grad == 0.0)
    assert ev.dsigma == pytest.approx(-1 / 0.5 + 0.4 ** 2 / 0.125, rel=1e-15)


# ----------------------------------------------------------- derivatives ----

def _richardson(f, v, h):
    d1 = (f(v + h) - f(v - h)) / (2 * h)
    d2 = (f(v + h / 2) - f(v - h / 2)) / h
    return (4 * d2 - d1) / 3


def test_gradient_vs_central_differences():
    x, y, mask = _rand_problem(40, 3, 0.6, 11, missing=0.15)
    sigma = 0.6
    ev = oracle.evaluate(x, y, sigma, mask)
    rng = np.random.default_rng(7)
    coords = [(int(i), int(k)) for i, k in zip(rng.integers(0, 40, 50), rng.integers(0, 3, 50))]
    for i, k in coords:
        def f(v, i=i, k=k):
            xx = x.copy()
            xx[i, k] = v
            return oracle.evaluate(xx, y, sigma, mask).loglik
        fd = _richardson(f, x[i, k], 1e-3)
        assert abs(fd - ev.grad[i, k]) <= 1e-8 * max(ev.absrow[i], 1.0), (i, k, fd, ev.grad[i, k])


def test_dsigma_vs_central_differences():
    x, y, mask = _rand_problem(30, 2, 0.4, 12, missing=0.1)
    for sigma in (0.05, 0.4, 3.0):
        ev = oracle.evaluate(x, y, sigma, mask)
        fd = _richardson(lambda s: oracle.evaluate(x, y, s, mask).loglik, sigma, sigma * 1e-3)
        assert abs(fd - ev.dsigma) <= 1e-8 * ev.abs_dsigma, (sigma, fd, ev.dsigma)


# ----------------------------------------------------------- invariances ----

def test_translation_invariance_rows_sum_to_zero():
    x, y, mask = _rand_problem(60, 2, 0.5, 13, missing=0.2)
    ev = oracle.evaluate(x, y, 0.5, mask)
    assert np.max(np.abs(ev.grad.sum(axis=0))) <= 1e-13 * ev.absrow.sum()
    ev2 = oracle.evaluate(x + np.array([3.0, -7.0]), y, 0.5, mask)
    assert _rel(ev2.loglik, ev.loglik, ev.abs_loglik) < 1e-13


def test_rotation_invariance_and_equivariance():
    x, y, mask = _rand_problem(50, 3, 0.8, 14)
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    ev = oracle.evaluate(x, y, 0.8, mask)
    evr = oracle.evaluate(x @ q, y, 0.8, mask)
    assert _rel(evr.loglik, ev.loglik, ev.abs_loglik) < 1e-13
    assert np.max(np.abs(evr.grad - ev.grad @ q)) <= 1e-12 * np.max(ev.absrow)
    # X^T G is symmetric (rotation invariance, infinitesimally)
    s = x.T @ ev.grad
    assert np.max(np.abs(s - s.T)) <= 1e-12 * np.max(np.abs(x)) * ev.absrow.sum()


def test_permutation_equivariance():
    x, y, mask = _rand_problem(30, 2, 0.7, 15, missing=0.2)
    perm = np.random.default_rng(4).permutation(30)
    ev = oracle.evaluate(x, y, 0.7, mask)
    evp = oracle.evaluate(x[perm], y[np.ix_(perm, perm)], 0.7, mask[np.ix_(perm, perm)])
    assert _rel(evp.loglik, ev.loglik, ev.abs_loglik) < 1e-13
    assert np.max(np.abs(evp.grad - ev.grad[perm])) <= 1e-13 * np.max(ev.absrow)


def test_scaling_identity_pins_log_sigma_term():
    # L(cX, cY, c sigma) = L(X, Y, sigma) - M ln c exactly
    x, y, mask = _rand_problem(25, 2, 0.5, 16, missing=0.1)
    ev = oracle.evaluate(x, y, 0.5, mask)
    for c in (0.1, 3.0, 17.0):
        evc = oracle.evaluate(c * x, c * y, c * 0.5, mask)
        assert _rel(evc.loglik, ev.loglik - ev.m_obs * math.log(c), ev.abs_loglik) < 1e-13
        # gradient scales as 1/c
        assert np.max(np.abs(evc.grad * c - ev.grad)) <= 1e-12 * np.max(ev.absrow)


def test_y_equal_delta_special_case():
    x, _, _ = _rand_problem(20, 2, 1.0, 17)
    from scipy.spatial.distance import cdist
    y = cdist(x, x)
    for sigma in (0.2, 1.0, 4.0):
        ev = oracle.evaluate(x, y, sigma)
        il = np.tril_indices(20, -1)
        ref = -np.sum(special.log_ndtr(y[il] / sigma)) - len(il[0]) * math.log(sigma)
        assert _rel(ev.loglik, ref, ev.abs_loglik) < 1e-13


def test_all_missing_gives_zero():
    x, y, _ = _rand_problem(10, 2, 1.0, 18)
    ev = oracle.evaluate(x, y, 0.4, np.ones((10, 10), np.uint8))
    assert ev.loglik == 0.0 and ev.dsigma == 0.0 and np.all(ev.grad == 0.0) and ev.m_obs == 0
    ev2 = oracle.evaluate(x, np.full((10, 10), np.nan), 0.4)
    assert ev2.loglik == 0.0 and ev2.m_obs == 0


def test_empty_and_single_point():
    ev = oracle.evaluate(np.zeros((1, 3)), np.zeros((1, 1)), 1.0)
    assert ev.loglik == 0.0 and np.all(ev.grad == 0)
    ev0 = oracle.evaluate(np.zeros((0, 2)), np.zeros((0, 0)), 1.0)
    assert ev0.loglik == 0.0 and ev0.grad.shape == (0, 2)


@pytest.mark.parametrize("delta,sigma", [(0.0, 1.0), (0.3, 0.5), (2.0, 1.0), (1.0, 0.2),
                                         (0.05, 2.0)])
def test_truncated_normal_density_integrates_to_one(delta, sigma):
    # For one pair, exp(L(y)) / sqrt(2 pi) is the density of y under Eq. (1):
    # it integrates to one over y > 0 only with Phi(+delta/sigma) in Eq. (2).
    x = np.array([[0.0], [delta]])

    def dens(v):
        y = np.array([[0.0, v], [v, 0.0]])
        return math.exp(oracle.evaluate(x, y, sigma).loglik) / math.sqrt(2 * math.pi)

    tot, err = integrate.quad(dens, 0, delta + 40 * sigma, points=[delta], limit=200)
    assert tot == pytest.approx(1.0, abs=1e-10)


# --------------------------------------------------------------- leapfrog ---

def _harmonic(x0, p0, lam, eps, steps):
    # with every pair missing the target is -lam/2 ||x||^2: the leapfrog map
    # of one step is linear, [x; p] <- A [x; p]
    a = np.array([[1 - eps * eps * lam / 2, eps],
                  [-eps * lam * (1 - eps * eps * lam / 4), 1 - eps * eps * lam / 2]])
    st = np.stack([x0.ravel(), p0.ravel()])
    for _ in range(steps):
        st = a @ st
    return st[0].reshape(x0.shape), st[1].reshape(p0.shape)


def test_leapfrog_harmonic_closed_form():
    rng = np.random.default_rng(20)
    x0 = rng.standard_normal((12, 2))
    p0 = rng.standard_normal((12, 2))
    y = np.ones((12, 12))
    mask = np.ones((12, 12), np.uint8)
    tr = oracle.leapfrog(x0, p0, y, 0.5, eps=0.1, n_steps=17, mask=mask, prior_precision=2.0)
    xr, pr = _harmonic(x0, p0, 2.0, 0.1, 17)
    assert np.max(np.abs(tr.x - xr)) < 1e-13
    assert np.max(np.abs(tr.p - pr)) < 1e-13


def test_leapfrog_single_step_by_hand():
    x, y, mask = _rand_problem(15, 2, 0.5, 21, missing=0.1)
    p = np.random.default_rng(5).standard_normal((15, 2))
    eps = 0.01
    g0 = oracle.evaluate(x, y, 0.5, mask).grad
    xh = x + eps * (p + 0.5 * eps * g0)
    g1 = oracle.evaluate(xh, y, 0.5, mask).grad
    ph = p + 0.5 * eps * g0 + 0.5 * eps * g1
    tr = oracle.leapfrog(x, p, y, 0.5, eps=eps, n_steps=1, mask=mask)
    assert np.allclose(tr.x, xh, rtol=0, atol=1e-15)
    assert np.allclose(tr.p, ph, rtol=0, atol=1e-13)
    assert np.allclose(tr.grad_end, g1, rtol=0, atol=1e-12)


def test_leapfrog_reversibility():
    x, y, mask = _rand_problem(30, 2, 0.8, 22, missing=0.1)
    p = np.random.default_rng(6).standard_normal((30, 2))
    fw = oracle.leapfrog(x, p, y, 0.8, eps=2e-3, n_steps=20, mask=mask, prior_precision=0.1)
    bw = oracle.leapfrog(fw.x, -fw.p, y, 0.8, eps=2e-3, n_steps=20, mask=mask,
                         prior_precision=0.1)
    assert np.max(np.abs(bw.x - x)) < 1e-12
    assert np.max(np.abs(-bw.p - p)) < 1e-11


def test_leapfrog_energy_error_is_second_order():
    x, y, mask = _rand_problem(30, 2, 0.8, 23)
    p = np.random.default_rng(8).standard_normal((30, 2))
    errs = []
    for eps in (4e-3, 2e-3, 1e-3):
        steps = int(round(0.08 / eps))
        tr = oracle.leapfrog(x, p, y, 0.8, eps=eps, n_steps=steps, mask=mask)
        errs.append(abs(tr.energy_end - tr.energy_start))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs


def test_leapfrog_unit_mass_matches_explicit_identity():
    x, y, mask = _rand_problem(12, 3, 0.5, 24)
    p = np.random.default_rng(9).standard_normal((12, 3))
    a = oracle.leapfrog(x, p, y, 0.5, eps=1e-3, n_steps=5)
    b = oracle.leapfrog(x, p, y, 0.5, eps=1e-3, n_steps=5, inv_mass=np.ones((12, 3)))
    assert np.array_equal(a.x, b.x) and np.array_equal(a.p, b.p)
    # a heavier mass on one coordinate slows its drift
    im = np.ones((12, 3))
    im[0, 0] = 0.0
    c = oracle.leapfrog(x, p, y, 0.5, eps=1e-3, n_steps=5, inv_mass=im)
    assert c.x[0, 0] == x[0, 0]


def test_grad_rows_vs_brute_force():
    # the per-row oracle (for sampled checks at large N) against mpmath
    x, y, mask = _rand_problem(8, 3, 0.4, 25, missing=0.2, nan_frac=0.1)
    ref = mpr.brute_force(x, y, 0.4, mask)
    rows = [0, 3, 7]
    g, a, b = oracle.grad_rows(x, y, 0.4, rows, mask)
    ev = oracle.evaluate(x, y, 0.4, mask)
    for r, i in enumerate(rows):
        gref = np.array([float(v) for v in ref["grad"][i]])
        assert np.max(np.abs(g[r] - gref)) <= 1e-14 * ev.absrow[i]
        assert a[r] == pytest.approx(float(ref["absrow"][i]), rel=1e-14)
        assert b[r] == pytest.approx(float(ref["condrow"][i]), rel=1e-14)


def test_grad_rows_given_vs_brute_force():
    # the same rows from whole rows of the symmetric Y (missing folded to NaN)
    x, y, mask = _rand_problem(9, 2, 0.6, 27, missing=0.2, nan_frac=0.1)
    ref = mpr.brute_force(x, y, 0.6, mask)
    yf = np.where(mask != 0, np.nan, y)
    rows = [8, 0, 4]
    g, a, b = oracle.grad_rows_given(x, yf[rows], 0.6, rows)
    ev = oracle.evaluate(x, y, 0.6, mask)
    for r, i in enumerate(rows):
        gref = np.array([float(v) for v in ref["grad"][i]])
        assert np.max(np.abs(g[r] - gref)) <= 1e-14 * ev.absrow[i]
        assert a[r] == pytest.approx(float(ref["absrow"][i]), rel=1e-14)
        assert b[r] == pytest.approx(float(ref["condrow"][i]), rel=1e-14)
    with pytest.raises(ValueError):
        oracle.grad_rows_given(x, yf[rows], 0.6, [0, 9, 1])


def test_row_rounding_scale_bounds_the_row():
    # B_i = sum (delta + |y|)/sigma^2 + m/sigma bounds every |w_ij|, so B_i >= A_i
    x, y, mask = _rand_problem(40, 2, 0.3, 26, missing=0.1)
    ev = oracle.evaluate(x, y, 0.3, mask)
    assert np.all(ev.condrow >= ev.absrow) and np.all(ev.absrow >= np.abs(ev.grad).max(axis=1))


# ------------------------------------------- model without truncation ----

def test_untruncated_against_normal_density():
    """The ablation model (no truncation to y > 0) against mpmath's normal
    density, with the gradient and sigma-derivative by numerical
    differentiation of that density."""
    rng = np.random.default_rng(77)
    n, d = 6, 2
    x = rng.standard_normal((n, d)) * 1.5
    y = np.abs(rng.standard_normal((n, n))) * 2 + 0.1
    y = np.tril(y, -1)
    y = y + y.T
    mask = np.zeros((n, n), np.uint8)
    mask[4, 1] = mask[1, 4] = 1
    y[5, 2] = y[2, 5] = np.nan
    ref = mpr.brute_force_normal(x, y, 0.8, mask)
    got = oracle.evaluate(x, y, 0.8, mask, truncated=False)
    assert got.m_obs == ref["m_obs"] == 13
    assert abs(got.loglik - float(ref["loglik"])) <= 1e-14 * abs(float(ref["loglik"]))
    g = np.array([[float(v) for v in row] for row in ref["grad"]])
    assert np.abs(got.grad - g).max() <= 1e-12 * np.abs(g).max()
    assert abs(got.dsigma - float(ref["dsigma"])) <= 1e-12 * abs(float(ref["dsigma"]))


def test_truncation_term_is_the_only_difference():
    rng = np.random.default_rng(78)
    n, d, sigma = 40, 3, 0.9
    x = rng.standard_normal((n, d)) * 2
    y = np.abs(rng.standard_normal((n, n))) * 3
    y = np.tril(y, -1)
    y = y + y.T
    a = oracle.evaluate(x, y, sigma)
    b = oracle.evaluate(x, y, sigma, truncated=False)
    i, j = np.tril_indices(n, -1)
    delta = np.sqrt(((x[i] - x[j]) ** 2).sum(1))
    lnphi = oracle.log_phi(delta / sigma)
    assert abs((b.loglik - a.loglik) - lnphi.sum()) <= 1e-12 * abs(a.loglik)
    assert a.m_obs == b.m_obs
    # the untruncated gradient has no phi/Phi term: its rows sum to zero too
    assert np.abs(b.grad.sum(0)).max() <= 1e-12 * np.abs(b.grad).max()


def test_untruncated_leapfrog_step_by_hand_and_order():
    """The leapfrog on the model without truncation: one step written out
    from the normal model's gradient (pinned above against mpmath), and the
    energy error of a trajectory falling as eps^2."""
    x, y, mask = _rand_problem(12, 2, 0.8, 31, missing=0.1)
    p = np.random.default_rng(5).standard_normal((12, 2))
    eps = 1e-3
    tr = oracle.leapfrog(x, p, y, 0.8, eps, 1, mask=mask, truncated=False)
    g0 = oracle.evaluate(x, y, 0.8, mask, truncated=False).grad
    ph = p + 0.5 * eps * g0
    x1 = x + eps * ph
    g1 = oracle.evaluate(x1, y, 0.8, mask, truncated=False).grad
    assert np.abs(tr.x - x1).max() <= 1e-15 * np.abs(x1).max()
    assert np.abs(tr.p - (ph + 0.5 * eps * g1)).max() <= 1e-13 * np.abs(p).max()
    # the truncated model's trajectory differs (the phi/Phi term acts)
    trt = oracle.leapfrog(x, p, y, 0.8, eps, 1, mask=mask)
    assert np.abs(trt.p - tr.p).max() > 1e-9
    errs = []
    for e in (4e-3, 2e-3, 1e-3):
        t = oracle.leapfrog(x, p, y, 0.8, e, int(round(0.04 / e)), mask=mask, truncated=False)
        errs.append(abs(t.energy_end - t.energy_start))
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_untruncated_hmc_step_is_its_leapfrog():
    # an accepted transition of the model without truncation ends where the
    # leapfrog from its momentum draw ends
    x, y, mask = _rand_problem(10, 2, 0.9, 32)
    st = oracle.hmc_step(x, y, 0.9, 1e-3, 5, seed=9, iteration=2, mask=mask, truncated=False)
    assert st.accepted
    mom = oracle.momentum(10, 2, 9, 2)
    tr = oracle.leapfrog(x, mom, y, 0.9, 1e-3, 5, mask=mask, truncated=False)
    assert np.array_equal(st.x, tr.x)
    assert st.loglik == tr.loglik_end


# --------------------------------------------- held-out predictive density ----

def _heldout_case(seed, n=7, d=2, frac=0.4):
    rng = np.random.default_rng(seed)
    y = np.abs(rng.standard_normal((n, n))) * 2 + 0.2
    y = np.tril(y, -1)
    y = y + y.T
    h = np.tril(rng.random((n, n)) < frac, -1)
    heldout = (h | h.T).astype(np.uint8)
    mask = np.zeros((n, n), np.uint8)
    i, j = np.nonzero(np.tril(heldout, -1))
    mask[i[0], j[0]] = mask[j[0], i[0]] = 1          # one held-out pair is missing
    return rng, y, heldout, mask


def test_lpd_against_mpmath_density():
    rng, y, heldout, mask = _heldout_case(5)
    xs = rng.standard_normal((4, 7, 2)) * 1.5
    sig = rng.uniform(0.5, 1.2, 4)
    ref, cnt = mpr.brute_force_lpd(xs, sig, y, heldout, mask)
    got, m = oracle.lpd(xs, sig, y, heldout, mask)
    assert m == cnt == int(np.tril(heldout, -1).sum()) - 1
    assert abs(got - float(ref)) <= 1e-13 * abs(float(ref))


def test_lpd_one_draw_is_the_likelihood_with_constant():
    """With one draw the lpd is the held-out problem's log-likelihood of
    Eq. (2) plus the 2 pi constant that Eq. (2) drops."""
    rng, y, heldout, mask = _heldout_case(6, n=30, d=3, frac=0.3)
    x = rng.standard_normal((30, 3)) * 2
    got, m = oracle.lpd(x, 0.8, y, heldout, mask)
    not_held = ((heldout == 0) | (mask != 0)).astype(np.uint8)
    ev = oracle.evaluate(x, y, 0.8, not_held)
    assert m == ev.m_obs
    assert abs(got - (ev.loglik - 0.5 * m * math.log(2 * math.pi))) <= 1e-12 * abs(got)


def test_lpd_draw_averaging():
    rng, y, heldout, _ = _heldout_case(7, n=20, d=2, frac=0.5)
    xs = rng.standard_normal((3, 20, 2)) * 2
    sig = np.array([0.7, 0.9, 1.1])
    a, _ = oracle.lpd(xs, sig, y, heldout)
    # repeating every draw leaves the average unchanged
    b, _ = oracle.lpd(np.concatenate([xs, xs]), np.concatenate([sig, sig]), y, heldout)
    assert abs(a - b) <= 1e-13 * abs(a)
    # Jensen: the log of the average is at least the average of the logs
    singles = [oracle.lpd(xs[s], sig[s], y, heldout)[0] for s in range(3)]
    assert a >= np.mean(singles) - 1e-12 * abs(a)
