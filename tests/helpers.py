"""Test-side helpers: closed forms, dense assembly and gauge transformations.

Nothing here implements the solver; the dense matrices are assembled column by
column from whichever operator is passed in, so that LAPACK can check it.
"""
from __future__ import annotations

import itertools

import numpy as np

import synth


def even_mask(L):
    return synth.site_parity(L) == 0


def to_even_vector(L, f):
    """Natural [V][3] field -> flat vector over (even site, colour)."""
    return np.asarray(f)[even_mask(L)].reshape(-1)


def from_even_vector(L, v):
    V = synth.volume(L)
    f = np.zeros((V, 3), np.complex128)
    f[even_mask(L)] = np.asarray(v).reshape(-1, 3)
    return f


def dense_even_operator(L, apply):
    """Dense matrix of an even->even operator given as a function of natural fields."""
    m = even_mask(L)
    n = int(m.sum()) * 3
    A = np.zeros((n, n), np.complex128)
    for j in range(n):
        e = np.zeros(n, np.complex128)
        e[j] = 1.0
        A[:, j] = to_even_vector(L, apply(from_even_vector(L, e)))
    return A


def free_spectrum(L, mass, antiperiodic=True, theta_t=0.0):
    """Closed-form eigenvalues of m^2 - D_eo D_oe for unit links (with multiplicity);
    theta_t: a constant U(1) phase on the time links (imaginary chemical
    potential), which shifts every time momentum by theta_t.

    Over the Brillouin zone the values m^2 + sum_mu sin^2 p_mu come in pairs
    (p, p + pi(1,1,1,1)) that share one even-site eigenvector, so each momentum
    pair contributes once, times 3 colours.
    """
    moms = []
    for mu, n in enumerate(L):
        if mu == 3 and antiperiodic:
            moms.append([(2 * k + 1) * np.pi / n + theta_t for k in range(n)])
        elif mu == 3:
            moms.append([2 * k * np.pi / n + theta_t for k in range(n)])
        else:
            moms.append([2 * k * np.pi / n for k in range(n)])
    vals = [mass ** 2 + sum(np.sin(p) ** 2 for p in ps) for ps in itertools.product(*moms)]
    vals = np.sort(np.array(vals))
    return np.repeat(vals[::2], 3)  # each value appears in pairs; keep one per pair


def plane_wave_even(L, p, colour_vec):
    """e^{i p.x} c on even sites, zero on odd sites."""
    X = synth.site_coords(L)
    ph = np.exp(1j * (X @ np.asarray(p, dtype=np.float64)))
    f = ph[:, None] * np.asarray(colour_vec)[None, :]
    f[~even_mask(L)] = 0
    return f


def neighbour_index(L, mu, direction=+1):
    X = synth.site_coords(L).copy()
    X[:, mu] = (X[:, mu] + direction) % L[mu]
    return X[:, 0] + L[0] * (X[:, 1] + L[1] * (X[:, 2] + L[2] * X[:, 3]))


def gauge_transform_links(L, U, g):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        fwd = neighbour_index(L, mu, +1)
        out[mu] = g @ U[mu] @ np.conj(np.swapaxes(g[fwd], -1, -2))
    return out


def gauge_transform_field(g, f):
    return np.einsum("xab,xb->xa", g, f)


def su3_exp(T):
    """exp(T) for anti-Hermitian T (stack), via eigendecomposition of -iT."""
    w, v = np.linalg.eigh(-1j * T)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def max_rel(a, b):
    """max |a - b| / max |b| over all complex entries."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
