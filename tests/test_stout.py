"""Oracle pins for stout smearing and its force chain rule (Sec. 2: the Dirac
operator uses k-times stout-smeared links; the MD force must be carried back
to the unsmeared links).  rho = 0 is the identity; smeared links are SU(3)
and gauge covariant; the chain rule is the derivative of a function of the
smeared links (central differences along random su(3) directions), for one
and for two levels."""
import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H


def test_rho_zero_is_identity_and_su3():
    L = (4, 4, 2, 4)
    U = synth.links_haar(L, 901)
    assert H.max_rel(oracle.stout_smear(L, U, 0.0), U) <= 1e-14
    S = oracle.stout_smear(L, U, 0.15)
    assert np.abs(S @ np.conj(np.swapaxes(S, -1, -2)) - np.eye(3)).max() <= 1e-13
    assert np.abs(np.linalg.det(S) - 1).max() <= 1e-13
    assert H.max_rel(S, U) > 1e-2


def test_gauge_covariance():
    L = (4, 2, 4, 4)
    U = synth.links_exp(L, 0.6, 902)
    g = synth.random_gauge_transform(L, 903)
    S1 = H.gauge_transform_links(L, oracle.stout_smear(L, U, 0.12), g)
    S2 = oracle.stout_smear(L, H.gauge_transform_links(L, U, g), 0.12)
    assert H.max_rel(S1, S2) <= 1e-13


@pytest.mark.parametrize("levels", [1, 2])
def test_chain_rule_is_derivative(levels):
    """S(U) = sum Re Tr[W U^(k)(U)] for a fixed W: dS/deps along U -> exp(eps T) U
    equals sum Tr[T F], F from the chain rule with G' = W^dag at the top."""
    L = (4, 2, 2, 4)
    rho = 0.1
    U = synth.links_exp(L, 0.5, 904)
    W = synth.gaussian_field(L, 12, 905).reshape(4, -1, 3, 3)

    def smear(Ux):
        for _ in range(levels):
            Ux = oracle.stout_smear(L, Ux, rho)
        return Ux

    def S(Ux):
        return float(np.real(np.einsum("...ab,...ba->...", W, smear(Ux)).sum()))

    chain = [U]
    for _ in range(levels - 1):
        chain.append(oracle.stout_smear(L, chain[-1], rho))
    G = np.conj(np.swapaxes(W, -1, -2))
    for j in range(levels - 1, -1, -1):
        G = oracle.stout_force(L, chain[j], rho, G, mode=0 if j == 0 else 1)
    F = G
    T = synth.su3_algebra_directions(L, 2, 906)
    eps = 1e-5
    for k in range(2):
        d = (S(H.su3_exp(eps * T[k]) @ U) - S(H.su3_exp(-eps * T[k]) @ U)) / (2 * eps)
        pred = float(np.real(np.einsum("...ab,...ba->...", T[k], F).sum()))
        assert abs(d - pred) <= 1e-7 * max(1.0, abs(pred))


@pytest.mark.parametrize("rho,mu", [(0.1, 0), (0.05, 3), (-0.07, 2)])
def test_single_link_weak_field_closed_form(rho, mu):
    """Unit links except one, U_mu(x0) = exp(eps T) (T traceless anti-Hermitian).
    Every staple of that link is then 1, so C = 6, Omega = 6 rho exp(-eps T),
    X = TA(Omega) = -6 rho eps T + O(eps^2) and the smeared link is
    exp((1 - 6 rho) eps T) + O(eps^2).  The central difference in eps gives
    the O(eps) coefficient (1 - 6 rho) T, which fixes the sign and the scale of
    rho (rho -> -rho gives 1 + 6 rho, rho / 2 gives 1 - 3 rho).  A link that
    shares no plaquette with x0 stays the identity exactly."""
    L = (4, 4, 4, 4)
    x0 = 37
    T = synth.su3_algebra_directions(L, 1, 911)[0, mu, x0]
    eps = 1e-4

    def smeared(e):
        U = synth.links_unit(L).copy()
        U[mu, x0] = H.su3_exp(e * T)
        return oracle.stout_smear(L, U, rho)

    Sp, Sm = smeared(eps), smeared(-eps)
    d = (Sp[mu, x0] - Sm[mu, x0]) / (2 * eps)
    assert np.abs(d - (1 - 6 * rho) * T).max() <= 1e-6 * np.abs(T).max()
    far = (x0 + 2 + 2 * L[0] + 2 * L[0] * L[1] + 2 * L[0] * L[1] * L[2]) % synth.volume(L)
    for nu in range(4):
        assert np.abs(Sp[nu, far] - np.eye(3)).max() == 0.0


def _mean_plaquette(L, U):
    """Mean over sites and the six planes of Re Tr P / 3, written out here."""
    tot = 0.0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            xm = H.neighbour_index(L, mu, +1)
            xn = H.neighbour_index(L, nu, +1)
            P = U[mu] @ U[nu][xm] @ np.conj(np.swapaxes(U[mu][xn], -1, -2)) \
                @ np.conj(np.swapaxes(U[nu], -1, -2))
            tot += np.real(np.trace(P, axis1=-2, axis2=-1)).mean() / 3
    return tot / 6


@pytest.mark.parametrize("gen", ["exp", "haar"])
def test_smearing_raises_the_plaquette(gen):
    """Stout smearing is a step of gradient flow of the Wilson action: for small
    positive rho the mean plaquette rises (and falls for rho < 0); a flipped
    sign of rho inverts both."""
    L = (4, 4, 4, 4)
    U = synth.links_exp(L, 0.6, 912) if gen == "exp" else synth.links_haar(L, 912)
    p0 = _mean_plaquette(L, U)
    assert _mean_plaquette(L, oracle.stout_smear(L, U, 0.1)) > p0 + 0.01
    assert _mean_plaquette(L, oracle.stout_smear(L, U, -0.1)) < p0 - 0.01
