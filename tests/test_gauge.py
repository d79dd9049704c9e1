"""Oracle pins for the gauge part of the MD (Sec. 2, Sec. 4.3): the tree-level
Symanzik action, its force and the momentum / link steps.

Closed forms: zero action and force on unit links; with a single non-unit
link V every loop through it has Re Tr = Re Tr V, and there are 6 plaquettes
and 18 rectangles through a link, so S = beta (1 - Re Tr V / 3)(6 c0 + 18 c1).
Exact symmetries: gauge invariance of S, covariance of F.  The force is the
derivative of the action (central differences along random su(3)
directions), and the MD steps conserve H = Tr H^2 / 2 + S to O(eps^2) with
leapfrog -- which fixes the sign convention between force and momentum."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H

C1 = -1.0 / 12.0


def _unit(L):
    V = int(np.prod(L))
    U = np.zeros((4, V, 3, 3), np.complex128)
    U[:, :] = np.eye(3)
    return U


@pytest.mark.parametrize("c1", [C1, 0.0])
def test_unit_links_zero_action_and_force(c1):
    L = (4, 4, 2, 6)
    U = _unit(L)
    assert oracle.gauge_action(L, U, 5.5, c1) == 0.0
    assert np.abs(oracle.gauge_force(L, U, 5.5, c1)).max() == 0.0


@pytest.mark.parametrize("c1", [C1, 0.0, 0.3])
@pytest.mark.parametrize("mu", [0, 3])
def test_single_link_closed_form(c1, mu):
    L = (4, 4, 4, 4)
    U = _unit(L)
    Vm = synth.haar_su3(synth.rng(5), 1)[0]
    U[mu, 37] = Vm
    beta = 4.2
    c0 = 1 - 8 * c1
    ref = beta * (1 - np.real(np.trace(Vm)) / 3) * (6 * c0 + 18 * c1)
    assert abs(oracle.gauge_action(L, U, beta, c1) - ref) <= 1e-12 * abs(ref)


def test_gauge_invariance_and_force_covariance():
    L = (4, 4, 4, 4)
    U = synth.links_exp(L, 0.6, 21)
    g = synth.random_gauge_transform(L, 22)
    Ug = H.gauge_transform_links(L, U, g)
    S, Sg = oracle.gauge_action(L, U, 3.3), oracle.gauge_action(L, Ug, 3.3)
    assert abs(S - Sg) <= 1e-12 * abs(S)
    F, Fg = oracle.gauge_force(L, U, 3.3), oracle.gauge_force(L, Ug, 3.3)
    ref = g[None] @ F @ np.conj(np.swapaxes(g, -1, -2))[None]
    assert H.max_rel(Fg, ref) <= 1e-12


@pytest.mark.parametrize("c1", [C1, 0.0])
def test_force_is_derivative_of_action(c1):
    """dS/deps along U -> exp(eps T) U equals sum Tr[T F] (central differences)."""
    L = (4, 4, 2, 4)
    U = synth.links_exp(L, 0.7, 23)
    beta = 3.1
    F = oracle.gauge_force(L, U, beta, c1)
    T = synth.su3_algebra_directions(L, 3, 24)
    eps = 1e-5
    for k in range(3):
        E_p, E_m = H.su3_exp(eps * T[k]), H.su3_exp(-eps * T[k])
        d = (oracle.gauge_action(L, E_p @ U, beta, c1) -
             oracle.gauge_action(L, E_m @ U, beta, c1)) / (2 * eps)
        pred = float(np.real(np.einsum("...ab,...ba->...", T[k], F).sum()))
        assert abs(d - pred) <= 1e-7 * max(1.0, abs(pred))


def test_force_is_traceless_antihermitian():
    L = (4, 2, 4, 4)
    F = oracle.gauge_force(L, synth.links_haar(L, 25), 2.0)
    assert np.abs(F + np.conj(np.swapaxes(F, -1, -2))).max() <= 1e-13
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() <= 1e-13


def test_md_links_exponential_is_su3():
    L = (2, 2, 2, 2)
    U = synth.links_haar(L, 26)
    Hm = synth.momenta(L, 27)
    assert np.abs(Hm - np.conj(np.swapaxes(Hm, -1, -2))).max() <= 1e-15
    assert np.abs(np.trace(Hm, axis1=-2, axis2=-1)).max() <= 1e-14
    U2 = oracle.md_links(U, Hm, 0.3)
    I = np.eye(3)
    assert np.abs(U2 @ np.conj(np.swapaxes(U2, -1, -2)) - I).max() <= 1e-13
    assert np.abs(np.linalg.det(U2) - 1).max() <= 1e-13
    # diagonal momentum: exp(i eps diag(h)) = diag(exp(i eps h))
    D = np.zeros_like(Hm)
    D[..., 0, 0], D[..., 1, 1], D[..., 2, 2] = 0.4, -0.1, -0.3
    E = oracle.md_links(_unit(L), D, 0.7)
    assert np.abs(E[..., 0, 0] - np.exp(0.28j)).max() <= 1e-15


def _leapfrog(L, U, Hm, beta, eps, nsteps):
    Hm = oracle.md_momenta(Hm, oracle.gauge_force(L, U, beta), eps / 2)
    for n in range(nsteps):
        U = oracle.md_links(U, Hm, eps)
        Hm = oracle.md_momenta(Hm, oracle.gauge_force(L, U, beta),
                               eps if n < nsteps - 1 else eps / 2)
    return U, Hm


def test_leapfrog_conserves_energy_to_second_order():
    L = (2, 2, 2, 4)
    beta = 5.0
    U0 = synth.links_exp(L, 0.5, 28)
    H0 = synth.momenta(L, 29)
    E0 = oracle.kinetic_energy(H0) + oracle.gauge_action(L, U0, beta)
    dE = []
    for n in (8, 16):
        U, Hm = _leapfrog(L, U0, H0, beta, 0.5 / n, n)
        dE.append(oracle.kinetic_energy(Hm) + oracle.gauge_action(L, U, beta) - E0)
    assert abs(dE[1]) < 1e-3 * E0
    assert 3.0 < dE[0] / dE[1] < 5.0   # O(eps^2); a wrong force sign breaks both
