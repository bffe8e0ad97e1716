"""High-precision brute force of the MDS likelihood, for pinning the oracle.

Written directly from the paper's formulas with mpmath's own special
functions (``mp.ncdf``, ``mp.npdf``), independently of the C oracle:
  * Eq. (2): L = -M ln sigma - sum_{i>j} [(y_ij - delta_ij)^2/(2 sigma^2)
    + ln Phi(delta_ij / sigma)]  (2*pi constant dropped);
  * Eq. (9): dL/dx_i = -sum_{j != i} [(delta_ij - y_ij)/sigma^2
    + phi(delta_ij/sigma)/(sigma Phi(delta_ij/sigma))] (x_i - x_j)/delta_ij;
  * dL/dsigma by direct differentiation of Eq. (2).
Only small N (pure-Python loops at 40 significant digits).
"""
from __future__ import annotations

import math

import mpmath as mp


def _observed(y, mask, i, j):
    if mask is not None and mask[i][j]:
        return False
    return not math.isnan(float(y[i][j]))


def brute_force(x, y, sigma, mask=None, dps=40, truncated=True):
    """L, dL/dX, dL/dsigma and the observed-pair count, plus the magnitude
    sums that scale the rounding error of each output (the same pair terms
    with every summand taken in absolute value):
      absrow[i]  = sum_j |w_ij|                                   (A_i)
      condrow[i] = sum_j [(delta_ij + |y_ij|)/sigma^2 + m_ij/sigma] (B_i, the
                   bracket w_ij with both of its terms' sizes added)
      abs_loglik = sum |r_ij| + M |ln sigma|
      abs_dsigma = sum |(y - delta)^2/sigma^3 + delta m/sigma^2| + M/sigma
    with m_ij = phi(t)/Phi(t).  truncated=False: the same sums with the ln Phi
    and phi/Phi terms left out (normal errors without the truncation)."""
    with mp.workdps(dps):
        n = len(x)
        d = len(x[0])
        s = mp.mpf(sigma)
        X = [[mp.mpf(float(v)) for v in row] for row in x]
        L = mp.mpf(0)
        dS = mp.mpf(0)
        absL = mp.mpf(0)
        absS = mp.mpf(0)
        G = [[mp.mpf(0)] * d for _ in range(n)]
        A = [mp.mpf(0)] * n
        B = [mp.mpf(0)] * n
        m = 0
        for i in range(n):
            for j in range(i):
                if not _observed(y, mask, i, j):
                    continue
                m += 1
                yij = mp.mpf(float(y[i][j]))
                diff = [X[i][k] - X[j][k] for k in range(d)]
                delta = mp.sqrt(mp.fsum(v * v for v in diff))
                t = delta / s
                Phi = mp.ncdf(t)
                phi = mp.npdf(t)
                # ln Phi(t) = log1p(-Phi(-t)) keeps every digit as Phi(t) -> 1
                lnPhi = mp.log1p(-mp.ncdf(-t)) if truncated else mp.mpf(0)
                mills = phi / Phi if truncated else mp.mpf(0)
                r = (yij - delta) ** 2 / (2 * s * s) + lnPhi
                L -= r
                absL += abs(r)
                w = (delta - yij) / (s * s) + mills / s
                A[i] += abs(w)
                A[j] += abs(w)
                b = (delta + abs(yij)) / (s * s) + mills / s
                B[i] += b
                B[j] += b
                if delta != 0:
                    for k in range(d):
                        G[i][k] -= w * diff[k] / delta
                        G[j][k] += w * diff[k] / delta
                ds = (yij - delta) ** 2 / s ** 3 + delta / (s * s) * mills
                dS += ds
                absS += abs(ds)
        if m:
            L -= m * mp.log(s)
            dS -= m / s
            absL += m * abs(mp.log(s))
            absS += m / s
        return dict(loglik=L, grad=G, dsigma=dS, m_obs=m, absrow=A, condrow=B,
                    abs_loglik=absL, abs_dsigma=absS)


def log_phi(t, dps=50):
    with mp.workdps(dps):
        t = mp.mpf(t)
        return mp.log1p(-mp.ncdf(-t)) if t > 0 else mp.log(mp.ncdf(t))


def mills(t, dps=50):
    with mp.workdps(dps):
        t = mp.mpf(t)
        return mp.npdf(t) / mp.ncdf(t)


def brute_force_normal(x, y, sigma, mask=None, dps=40):
    """The untruncated model (plain normal errors) from mpmath's normal
    density: L = sum_{observed i>j} [ln N(y_ij; delta_ij, sigma^2) + ln sqrt(2 pi)]
    (the same 2*pi constant dropped as in Eq. 2); its gradient and
    sigma-derivative by mpmath's numerical differentiation of that L."""
    with mp.workdps(dps):
        n = len(x)
        d = len(x[0])
        pairs = [(i, j, mp.mpf(float(y[i][j]))) for i in range(n) for j in range(i)
                 if _observed(y, mask, i, j)]

        def loglik(flat, s):
            tot = mp.mpf(0)
            for i, j, yij in pairs:
                delta = mp.sqrt(mp.fsum((flat[i * d + k] - flat[j * d + k]) ** 2
                                        for k in range(d)))
                tot += mp.log(mp.npdf(yij, delta, s)) + mp.log(mp.sqrt(2 * mp.pi))
            return tot

        flat = [mp.mpf(float(v)) for row in x for v in row]
        s = mp.mpf(sigma)
        L = loglik(flat, s)
        G = []
        for c in range(n * d):
            def f(v, c=c):
                g = list(flat)
                g[c] = v
                return loglik(g, s)
            G.append(mp.diff(f, flat[c]))
        dS = mp.diff(lambda v: loglik(flat, v), s)
        return dict(loglik=L, grad=[G[i * d:(i + 1) * d] for i in range(n)], dsigma=dS,
                    m_obs=len(pairs))


def brute_force_lpd(xs, sigmas, y, heldout, mask=None, dps=40):
    """Log pointwise predictive density from mpmath's normal density and
    normal CDF: for each held-out observed pair, ln of the average over the
    draws of npdf(y; delta, sigma) / ncdf(delta / sigma)."""
    with mp.workdps(dps):
        n = len(xs[0])
        d = len(xs[0][0])
        tot = mp.mpf(0)
        cnt = 0
        for i in range(n):
            for j in range(i):
                if not heldout[i][j] or not _observed(y, mask, i, j):
                    continue
                dens = []
                for x, s in zip(xs, sigmas):
                    s = mp.mpf(float(s))
                    delta = mp.sqrt(mp.fsum((mp.mpf(float(x[i][k])) - mp.mpf(float(x[j][k]))) ** 2
                                            for k in range(d)))
                    dens.append(mp.npdf(mp.mpf(float(y[i][j])), delta, s) / mp.ncdf(delta / s))
                tot += mp.log(mp.fsum(dens) / len(dens))
                cnt += 1
        return tot, cnt
