"""Seeded synthetic inputs for the staggered even/odd solver.

This module is shared by the CPU oracle tests, the GPU parity tests, the
benchmark and the smoke check.  It holds no arithmetic of the method itself
(no hopping term, no solver, no force): it only draws gauge links, sources,
gauge transformations and su(3) directions from a seeded PCG64 stream, and
fixes the lattice geometry conventions (site ordering, parity) that both sides
must agree on as an input format.

Conventions
-----------
* A lattice has extents ``L = (Lx, Ly, Lz, Lt)``; direction mu = 0, 1, 2, 3 is
  x, y, z, t.  The lexicographic site index is
  ``lex = x + Lx*(y + Ly*(z + Lz*t))`` (x fastest).
* The parity of a site is ``(x + y + z + t) % 2``; 0 is even.
* Natural gauge field: complex128 array ``[4][V][3][3]``, ``U[mu, lex, a, b]``
  is row a, column b of the link leaving site lex in direction mu.
* Natural colour vector field: complex128 ``[V][3]`` (or ``[n][V][3]``).

The paper (Sec. 2) only states that links are SU(3) matrices; the
distributions below are the synthetic stand-ins for its thermalised
production configurations, which are not available.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

__all__ = [
    "volume", "site_coords", "site_parity", "rng",
    "links_unit", "links_exp", "links_haar", "haar_su3",
    "gaussian_field", "gaussian_even_source", "su3_algebra_directions",
    "su3_algebra_coeffs", "su3_from_coeffs", "expi_coeffs",
    "rational_shifts", "rational_weights",
]


def volume(L) -> int:
    L = tuple(int(v) for v in L)
    return L[0] * L[1] * L[2] * L[3]


def site_coords(L) -> np.ndarray:
    """Coordinates ``[V][4]`` (x, y, z, t) of every site in lexicographic order."""
    Lx, Ly, Lz, Lt = (int(v) for v in L)
    t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly),
                             np.arange(Lx), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def site_parity(L) -> np.ndarray:
    """Parity ``[V]`` (0 even, 1 odd) of every site in lexicographic order."""
    return site_coords(L).sum(axis=1) % 2


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _complex_gauss(g: np.random.Generator, shape) -> np.ndarray:
    """Complex Gaussian with E|z|^2 = 1: (N(0,1) + i N(0,1)) / sqrt(2)."""
    re = g.standard_normal(shape)
    im = g.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def links_unit(L) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    V = volume(L)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def _gell_mann() -> np.ndarray:
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j; lam[1][1, 0] = 1j
    lam[2][0, 0] = 1; lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j; lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j; lam[6][2, 1] = 1j
    lam[7][0, 0] = lam[7][1, 1] = 1 / np.sqrt(3); lam[7][2, 2] = -2 / np.sqrt(3)
    return lam


def _gaussian_hermitian(g: np.random.Generator, n: int) -> np.ndarray:
    """n traceless Hermitian 3x3 matrices H = sum_a c_a lambda_a / 2, c_a ~ N(0,1)."""
    c = g.standard_normal((n, 8))
    return np.einsum("na,aij->nij", c, _gell_mann() / 2.0)


_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "synth_gen.c")
_GEN_LIB = os.path.join(_HERE, "libsynth_gen.so")
_gen = None
_CHUNK = 1 << 21


def build(force: bool = True) -> str:
    """Compile the generator helper (gcc, OpenMP)."""
    if force or not os.path.exists(_GEN_LIB) or os.path.getmtime(_GEN_LIB) < os.path.getmtime(_GEN_SRC):
        tmp = _GEN_LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o",
                               tmp, _GEN_SRC, "-lm"])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _lib():
    global _gen
    if _gen is None:
        build(force=False)
        lib = ctypes.CDLL(_GEN_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.synth_su3_from_gauss.argtypes = [dp, dp, ctypes.c_long]
        lib.synth_su3_expi.argtypes = [dp, ctypes.c_double, dp, ctypes.c_long]
        _gen = lib
    return _gen


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def links_exp(L, beta: float, seed: int) -> np.ndarray:
    """Near-unit SU(3) links exp(i*beta*H), H = sum_a c_a lambda_a / 2 with
    c_a ~ N(0,1) (Gaussian traceless Hermitian).  The exponential is taken by
    scaling and squaring in the C helper, rows re-orthonormalised to SU(3)."""
    V = volume(L)
    g = rng(seed)
    out = np.empty((4 * V, 3, 3), np.complex128)
    for lo in range(0, 4 * V, _CHUNK):
        hi = min(4 * V, lo + _CHUNK)
        c = np.ascontiguousarray(g.standard_normal((hi - lo, 8)))
        _lib().synth_su3_expi(_dp(c), float(beta), _dp(out[lo:hi]), hi - lo)
    return out.reshape(4, V, 3, 3)


def haar_su3(g: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(3) matrices.

    Rows 0 and 1 are Gram-Schmidt orthonormalised complex Gaussian vectors
    (the first two rows of a Haar U(3) matrix); row 2 = conj(row0 x row1)
    fixes det = 1.  Completing the rows this way commutes with right
    multiplication by SU(3) (Z -> Z V), so the result is right-invariant, i.e. Haar on SU(3).
    """
    out = np.empty((n, 3, 3), np.complex128)
    for lo in range(0, n, _CHUNK):
        hi = min(n, lo + _CHUNK)
        # interleaved (re, im) standard normals; Gram-Schmidt ignores the scale
        z = g.standard_normal((hi - lo, 18))
        _lib().synth_su3_from_gauss(_dp(z), _dp(out[lo:hi]), hi - lo)
    return out


def links_haar(L, seed: int) -> np.ndarray:
    V = volume(L)
    return haar_su3(rng(seed), 4 * V).reshape(4, V, 3, 3)


def gaussian_field(L, n: int, seed: int) -> np.ndarray:
    """n complex Gaussian colour-vector fields on all sites, ``[n][V][3]``."""
    return _complex_gauss(rng(seed), (n, volume(L), 3))


def gaussian_even_source(L, n: int, seed: int) -> np.ndarray:
    """n Gaussian sources living on even sites (odd sites are zero), ``[n][V][3]``."""
    f = gaussian_field(L, n, seed)
    f[:, site_parity(L) == 1, :] = 0.0
    return f


def su3_algebra_coeffs(L, n: int, seed: int) -> np.ndarray:
    """Gell-Mann coefficients ``[n][4][V][8]`` (N(0,1)) of n random su(3)
    directions, one traceless anti-Hermitian T = i sum_a c_a lambda_a / 2 per link."""
    return rng(seed).standard_normal((n, 4, volume(L), 8))


def su3_from_coeffs(c: np.ndarray) -> np.ndarray:
    """T = i sum_a c_a lambda_a / 2 for coefficient arrays ``[..., 8]``."""
    return 1j * np.einsum("...a,aij->...ij", c, _gell_mann() / 2.0)


def expi_coeffs(c: np.ndarray, beta: float) -> np.ndarray:
    """exp(beta T) = exp(i beta sum_a c_a lambda_a / 2) for coefficients ``[..., 8]``."""
    c2 = np.ascontiguousarray(c, dtype=np.float64).reshape(-1, 8)
    out = np.empty((c2.shape[0], 3, 3), np.complex128)
    for lo in range(0, c2.shape[0], _CHUNK):
        hi = min(c2.shape[0], lo + _CHUNK)
        _lib().synth_su3_expi(_dp(c2[lo:hi]), float(beta), _dp(out[lo:hi]), hi - lo)
    return out.reshape(c.shape[:-1] + (3, 3))


def su3_algebra_directions(L, n: int, seed: int) -> np.ndarray:
    """n random su(3) directions, one traceless anti-Hermitian matrix per link.

    Shape ``[n][4][V][3][3]``; each matrix is i * sum_a c_a lambda_a / 2 with the
    coefficients of su3_algebra_coeffs(L, n, seed).
    """
    return su3_from_coeffs(su3_algebra_coeffs(L, n, seed))


def momenta(L, seed: int) -> np.ndarray:
    """Gaussian MD momenta, one traceless Hermitian matrix per link ``[4][V][3][3]``
    with density exp(-Tr H^2 / 2): H = sum_a c_a lambda_a / sqrt(2), c_a ~ N(0, 1)
    (Tr lambda_a lambda_b = 2 delta_ab)."""
    c = rng(seed).standard_normal((4, volume(L), 8))
    return np.einsum("...a,aij->...ij", c, _gell_mann() / np.sqrt(2.0))


def u1_phases_chemical(L, mu_i: float) -> np.ndarray:
    """theta_mu(x) ``[4][V]`` of a constant imaginary chemical potential: mu_i
    on every time link, zero elsewhere (u_t(x) = exp(i mu_i))."""
    th = np.zeros((4, volume(L)))
    th[3] = float(mu_i)
    return th


def u1_phases_magnetic(L, b: int) -> np.ndarray:
    """theta_mu(x) ``[4][V]`` of a uniform field along z with b flux quanta
    through the x-y plane (Landau gauge, periodic): theta_y = 2 pi b x /
    (Lx Ly) on y links; theta_x = -2 pi b y / Ly on the x links leaving
    x = Lx - 1.  Every x-y plaquette carries the phase 2 pi b / (Lx Ly)."""
    c = site_coords(L)
    th = np.zeros((4, volume(L)))
    th[1] = 2 * np.pi * b * c[:, 0] / (L[0] * L[1])
    th[0] = np.where(c[:, 0] == L[0] - 1, -2 * np.pi * b * c[:, 1] / L[1], 0.0)
    return th


def u1_phases_pure_gauge(L, seed: int):
    """(theta, alpha): theta_mu(x) = alpha(x + mu) - alpha(x) for a random
    alpha(x) in [0, 2 pi) -- a U(1) gauge transformation in phase form."""
    alpha = rng(seed).uniform(0, 2 * np.pi, volume(L))
    c = site_coords(L)
    th = np.zeros((4, volume(L)))
    for mu in range(4):
        cf = c.copy()
        cf[:, mu] = (cf[:, mu] + 1) % L[mu]
        lex = cf[:, 0] + L[0] * (cf[:, 1] + L[1] * (cf[:, 2] + L[2] * cf[:, 3]))
        th[mu] = alpha[lex] - alpha
    return th, alpha


def random_gauge_transform(L, seed: int) -> np.ndarray:
    """A Haar SU(3) matrix per site, ``[V][3][3]``."""
    return haar_su3(rng(seed), volume(L))


def rational_shifts(n: int = 12, lo: float = 1e-4, hi: float = 10.0) -> np.ndarray:
    """Pole positions sigma_k, log-spaced and inclusive on [lo, hi]."""
    return np.logspace(np.log10(lo), np.log10(hi), n)


def rational_weights(sigma: np.ndarray) -> np.ndarray:
    """Residues alpha_k for a stand-in rational form of x^(-1/4).

    The paper does not print its coefficients.  This uses the integral
    x^(-1/4) = sin(pi/4)/pi * int_0^inf t^(-1/4) / (t + x) dt discretised on
    the same logarithmic grid as the poles, so alpha_k = sin(pi/4)/pi *
    sigma_k^(3/4) * Delta with Delta the log-grid step.  Every check that
    uses them holds for any positive alpha.
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.size < 2:
        return np.ones_like(sigma)
    delta = np.log(sigma[-1] / sigma[0]) / (sigma.size - 1)
    return np.sin(np.pi / 4) / np.pi * sigma ** 0.75 * delta
