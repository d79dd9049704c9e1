"""Oracle pins for the U(1) phases on the links (Sec. 4.1): the Dirac operator
hops with u_mu(x) U_mu(x), u = exp(i theta_mu(x)).

Closed form: a constant phase theta on the time links (imaginary chemical
potential) shifts every time momentum of the free field by theta.  Exact
symmetries: a pure-gauge phase theta_mu(x) = alpha(x+mu) - alpha(x) is a U(1)
gauge transformation, D[u U] e^{-i alpha} psi = e^{-i alpha} D[U] psi; D_oe^dag
= -D_eo still holds; the magnetic-field generator puts the same flux through
every x-y plaquette."""
import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H


def _unit(L):
    U = np.zeros((4, int(np.prod(L)), 3, 3), np.complex128)
    U[:, :] = np.eye(3)
    return U


@pytest.mark.parametrize("L,mu_i", [((4, 4, 4, 4), 0.3), ((2, 4, 2, 6), 0.9), ((4, 2, 2, 4), -1.3)])
@pytest.mark.parametrize("anti", [True, False])
def test_imaginary_chemical_potential_free_spectrum(L, mu_i, anti):
    m = 0.2
    Up = oracle.phase_links(_unit(L), synth.u1_phases_chemical(L, mu_i))
    A = H.dense_even_operator(L, lambda f: oracle.apply_A(L, Up, m, 0.0, f, anti))
    lam = np.sort(np.linalg.eigvalsh(A))
    ref = H.free_spectrum(L, m, anti, theta_t=mu_i)
    assert np.allclose(lam, ref, rtol=0, atol=1e-12)
    # and the phase matters: without it the spectrum differs
    assert not np.allclose(lam, H.free_spectrum(L, m, anti), rtol=0, atol=1e-6)


def test_pure_gauge_phase_is_a_gauge_transformation():
    L = (4, 4, 2, 4)
    U = synth.links_haar(L, 701)
    th, alpha = synth.u1_phases_pure_gauge(L, 702)
    psi = synth.gaussian_even_source(L, 1, 703)[0]
    lam = np.exp(-1j * alpha)[:, None]  # u U = e^{-i alpha(x)} U e^{i alpha(x+mu)}
    got = oracle.doe(L, oracle.phase_links(U, th), lam * psi)
    ref = lam * oracle.doe(L, U, psi)
    assert H.max_rel(got, ref) <= 1e-13


def test_phased_operator_keeps_anti_hermiticity():
    L = (4, 4, 4, 2)
    U = oracle.phase_links(synth.links_haar(L, 704), synth.u1_phases_magnetic(L, 3) +
                           synth.u1_phases_chemical(L, 0.4))
    e = synth.gaussian_even_source(L, 1, 705)[0]
    o = synth.gaussian_field(L, 1, 706)[0]
    o[synth.site_parity(L) == 0] = 0
    lhs = np.vdot(o, oracle.doe(L, U, e))
    rhs = -np.vdot(oracle.deo(L, U, o), e)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("L,b", [((4, 6, 2, 2), 1), ((6, 4, 2, 2), 5)])
def test_magnetic_phases_uniform_flux(L, b):
    th = synth.u1_phases_magnetic(L, b)
    c = synth.site_coords(L)

    def lex(cc):
        return cc[:, 0] + L[0] * (cc[:, 1] + L[1] * (cc[:, 2] + L[2] * cc[:, 3]))

    cx, cy = c.copy(), c.copy()
    cx[:, 0] = (cx[:, 0] + 1) % L[0]
    cy[:, 1] = (cy[:, 1] + 1) % L[1]
    flux = th[0] + th[1][lex(cx)] - th[0][lex(cy)] - th[1]
    assert np.allclose(np.exp(1j * flux), np.exp(2j * np.pi * b / (L[0] * L[1])), atol=1e-12)
