"""Rational approximations of the fractional powers used by RHMC.

RHMC replaces a fractional power of the even/odd operator A = m^2 - D_eo D_oe
by a rational function of A, approximated to machine precision, whose poles
are the shifts sigma_i of the multi-shift solves (Sec. 2, Eq. (2)).  In
partial fractions

    r(x) = alpha0 + sum_i alpha_i / (x + sigma_i),

so r(A) b = alpha0 b + sum_i alpha_i (A + sigma_i)^-1 b needs one multi-shift
solve and one linear combination.

`minimax` computes the best uniform relative-error approximation of x**p of
type (n, n) on a spectral interval [lo, hi] with the Remez exchange
algorithm: on a reference of 2n + 2 points the rational function with
equal, alternating relative errors is found from a linear system (the level
E enters multiplied by the previous denominator, and the system is solved
again until E settles); the reference then moves to the 2n + 2 alternating
extrema of the error, until the extrema are equal.  The reference systems
are Vandermonde-like and badly conditioned over several decades, so they are
solved in multiprecision arithmetic (mpmath) in the scaled variable
y = x / sqrt(lo hi); the partial fractions come from the roots of the
denominator and the residues N(y_i) / D'(y_i).  Host-side setup, computed
once per (power, interval, degree).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = ["RationalApprox", "minimax", "minimax_for_tol", "spectral_bounds"]


@dataclass(frozen=True)
class RationalApprox:
    """r(x) = alpha0 + sum_i alpha[i] / (x + sigma[i]) ~ x**power on [lo, hi]."""
    power: float
    lo: float
    hi: float
    alpha0: float
    alpha: np.ndarray
    sigma: np.ndarray
    max_rel_error: float   # max |r(x) / x**power - 1| over [lo, hi]
    min_extremum: float    # smallest |error| at the 2n + 2 alternating extrema
    iterations: int

    @property
    def degree(self) -> int:
        return len(self.sigma)

    def __call__(self, x):
        x = np.asarray(x, dtype=np.float64)
        return self.alpha0 + np.sum(self.alpha / (x[..., None] + self.sigma), axis=-1)


def spectral_bounds(mass: float) -> tuple[float, float]:
    """Interval holding the spectrum of A = m^2 - D_eo D_oe for unitary links:
    -D_eo D_oe = D_oe^dagger D_oe >= 0, and every hop of D carries a factor
    1/2 and a unitary link, so |D| <= 4 and the spectrum lies in [m^2, m^2 + 16]."""
    m2 = float(mass) ** 2
    return m2, m2 + 16.0


def _rel_error(alpha0, alpha, sigma, p, x):
    r = alpha0 + np.sum(alpha / (x[:, None] + sigma), axis=1)
    return r * np.power(x, -p) - 1.0


def _alternating_extrema(x, e, npts):
    """Indices of npts extrema of e on the grid x with alternating signs, or None."""
    a = np.abs(e)
    n = len(e)
    idx = [0]
    for i in range(1, n - 1):
        if a[i] >= a[i - 1] and a[i] >= a[i + 1]:
            idx.append(i)
    idx.append(n - 1)
    # one extremum per run of equal sign: the largest
    keep = []
    for i in idx:
        if keep and np.sign(e[i]) == np.sign(e[keep[-1]]):
            if a[i] > a[keep[-1]]:
                keep[-1] = i
        else:
            keep.append(i)
    while len(keep) > npts:  # drop the smaller end extremum
        if a[keep[0]] < a[keep[-1]]:
            keep.pop(0)
        else:
            keep.pop()
    return keep if len(keep) == npts else None


def _refine(f, a, b, it=60):
    """Golden-section maximum of |f| on [a, b] (log variable)."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = abs(f(c)), abs(f(d))
    for _ in range(it):
        if fc > fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = abs(f(c))
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = abs(f(d))
        if b - a < 1e-13 * max(1.0, abs(a)):
            break
    return (a + b) / 2.0


def minimax(power: float, lo: float, hi: float, n: int, max_iter: int = 60,
            grid_per_point: int = 400) -> RationalApprox:
    """Best type-(n, n) relative-error approximation of x**power on [lo, hi].

    power in (-1, 1) and non-zero, 0 < lo < hi, 1 <= n <= 32.  Raises
    RuntimeError if the exchange does not reach equal extrema (to 0.1 %).
    """
    import mpmath

    p = float(power)
    if not (-1.0 < p < 1.0) or p == 0.0:
        raise ValueError(f"power must be in (-1, 1) and non-zero, got {power}")
    if not (0.0 < lo < hi) or not math.isfinite(hi):
        raise ValueError(f"need 0 < lo < hi, got [{lo}, {hi}]")
    if not (1 <= n <= 32):
        raise ValueError(f"degree must be in [1, 32], got {n}")
    xs = math.sqrt(lo * hi)
    u0, u1 = math.log(lo / xs), math.log(hi / xs)
    npts = 2 * n + 2
    kappa = hi / lo
    dps = 30 + int(math.ceil(0.6 * n * math.log10(kappa))) + 2 * n
    # scaled problem: g(y) = y**p on [lo/xs, hi/xs]; x**p = xs**p g(x/xs)
    ref = [math.exp(u0 + (u1 - u0) * (1.0 - math.cos(math.pi * k / (npts - 1))) / 2.0)
           for k in range(npts)]
    grid = np.exp(np.linspace(u0, u1, grid_per_point * npts))

    best = None
    with mpmath.workdps(dps):
        mpf = mpmath.mpf
        py = mpf(p)
        dold = None  # previous denominator (callable), None = 1
        for it in range(1, max_iter + 1):
            yk = [mpf(y) for y in ref]
            fk = [y ** py for y in yk]
            E = mpf(0)
            for inner in range(8):
                dk = [dold(y) if dold else mpf(1) for y in yk]
                M = mpmath.matrix(npts, npts)
                rhs = mpmath.matrix(npts, 1)
                for k in range(npts):
                    pw = [mpf(1)]
                    for _ in range(n):
                        pw.append(pw[-1] * yk[k])
                    for j in range(n + 1):
                        M[k, j] = pw[j]
                    for j in range(1, n + 1):
                        M[k, n + j] = -fk[k] * pw[j]
                    M[k, 2 * n + 1] = -(1 if k % 2 == 0 else -1) * fk[k] * dk[k]
                    rhs[k] = fk[k]
                sol = mpmath.lu_solve(M, rhs)
                c = [sol[j] for j in range(n + 1)]
                d = [mpf(1)] + [sol[n + j] for j in range(1, n + 1)]
                E_new = sol[2 * n + 1]

                def dnew(y, d=d):
                    return mpmath.polyval(d[::-1], y)

                dold = dnew
                done = abs(E_new - E) <= mpf("1e-6") * abs(E_new)
                E = E_new
                if done:
                    break
            # partial fractions from the roots of the denominator
            roots = mpmath.polyroots(d[::-1], maxsteps=400, extraprec=2 * dps)
            if any(abs(mpmath.im(r)) > mpf(10) ** (-dps // 3) * (1 + abs(r)) for r in roots):
                raise RuntimeError("Remez: complex poles (the exchange did not converge)")
            roots = sorted(mpmath.re(r) for r in roots)
            dprime = [j * d[j] for j in range(1, n + 1)]
            a0 = c[n] / d[n]
            res = [mpmath.polyval(c[::-1], r) / mpmath.polyval(dprime[::-1], r) for r in roots]
            s_y = [-r for r in roots]
            if any(s <= 0 for s in s_y):
                raise RuntimeError("Remez: a pole on the positive axis")
            scale = mpf(xs) ** py
            alpha0 = float(scale * a0)
            alpha = np.array([float(scale * mpf(xs) * a) for a in res])
            sigma = np.array([float(mpf(xs) * s) for s in s_y])

            # error of the double-precision partial fractions on the x axis
            xg = grid * xs
            eg = _rel_error(alpha0, alpha, sigma, p, xg)
            keep = _alternating_extrema(xg, eg, npts)
            if keep is None:
                raise RuntimeError(f"Remez: {npts} alternating extrema not found (degree {n})")

            def err_at(u):
                x = np.array([xs * math.exp(u)])
                return float(_rel_error(alpha0, alpha, sigma, p, x)[0])

            ug = np.log(grid)
            new_ref, vals = [], []
            for q, i in enumerate(keep):
                if i == 0 or i == len(grid) - 1:
                    u = ug[i]
                else:
                    u = _refine(err_at, ug[i - 1], ug[i + 1])
                new_ref.append(math.exp(u))
                vals.append(abs(err_at(u)))
            emax = max(max(vals), float(np.max(np.abs(eg))))
            emin = min(vals)
            best = RationalApprox(p, float(lo), float(hi), alpha0, alpha, sigma, emax, emin, it)
            if emax - emin <= 1e-3 * emax + 1e-15:
                return best
            ref = new_ref
    raise RuntimeError(f"Remez: no equioscillation after {max_iter} exchanges "
                       f"(max {best.max_rel_error:.3e}, min extremum {best.min_extremum:.3e})")


def minimax_for_tol(power: float, lo: float, hi: float, tol: float,
                    n_max: int = 32) -> RationalApprox:
    """Smallest-degree minimax approximation with max relative error <= tol."""
    if not (tol > 0.0):
        raise ValueError("tol must be positive")
    for n in range(1, n_max + 1):
        r = minimax(power, lo, hi, n)
        if r.max_rel_error <= tol:
            return r
    raise RuntimeError(f"no degree <= {n_max} reaches {tol:g} for x**{power} on [{lo}, {hi}]")
