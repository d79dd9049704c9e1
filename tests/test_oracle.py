"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Each test pins one part of the oracle to something other than itself:
closed-form spectra, exact symmetries, LAPACK dense solves, and finite
differences of the action.  A dropped term, a wrong sign, a wrong neighbour or
a transposed link in the oracle fails at least one of them.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H

LATTICES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 4), (2, 4, 2, 6)]


@pytest.fixture(scope="module", autouse=True)
def _build():
    oracle.build(force=False)


# ---------------------------------------------------------------- inputs

@pytest.mark.parametrize("gen", ["exp", "haar"])
def test_generated_links_are_su3(gen):
    L = (4, 4, 2, 2)
    U = synth.links_exp(L, 0.5, 7) if gen == "exp" else synth.links_haar(L, 7)
    I = np.eye(3)
    UU = U @ np.conj(np.swapaxes(U, -1, -2))
    assert np.max(np.abs(UU - I)) < 1e-13
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-13
    # same seed, same links
    U2 = synth.links_exp(L, 0.5, 7) if gen == "exp" else synth.links_haar(L, 7)
    assert np.array_equal(U, U2)


def test_third_row_is_conjugate_cross_product():
    """Sec. 4.1: for SU(3), r3 = (r1 x r2)^*; the 12-real link format relies on it."""
    U = synth.links_haar((4, 4, 4, 4), 3).reshape(-1, 3, 3)
    r3 = np.conj(np.cross(U[:, 0, :], U[:, 1, :]))
    assert np.max(np.abs(r3 - U[:, 2, :])) < 1e-14


# ---------------------------------------------------------------- hopping term

@pytest.mark.parametrize("L", LATTICES)
@pytest.mark.parametrize("anti", [True, False])
def test_doe_is_minus_deo_dagger(L, anti):
    """Sec. 2: D_oe^dag = -D_eo, checked as <chi, D_oe psi> = -<D_eo chi, psi>."""
    U = synth.links_haar(L, 11)
    par = synth.site_parity(L)
    psi = synth.gaussian_field(L, 1, 12)[0]
    psi[par == 1] = 0
    chi = synth.gaussian_field(L, 1, 13)[0]
    chi[par == 0] = 0
    lhs = np.vdot(chi, oracle.doe(L, U, psi, anti))
    rhs = -np.vdot(oracle.deo(L, U, chi, anti), psi)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("L", LATTICES)
def test_output_parity_and_input_parity(L):
    """D_oe writes only odd sites and reads only even sites (and vice versa)."""
    U = synth.links_exp(L, 0.3, 5)
    par = synth.site_parity(L)
    psi = synth.gaussian_field(L, 1, 6)[0]
    out = oracle.doe(L, U, psi)
    assert np.all(out[par == 0] == 0)
    psi_odd_garbage = psi.copy()
    psi_odd_garbage[par == 1] = 1e6
    assert np.array_equal(oracle.doe(L, U, psi_odd_garbage), out)
    out2 = oracle.deo(L, U, psi)
    assert np.all(out2[par == 1] == 0)


@pytest.mark.parametrize("L,anti", [((4, 4, 4, 4), True), ((4, 4, 4, 4), False),
                                    ((2, 4, 6, 4), True), ((6, 2, 4, 2), True)])
def test_free_field_spectrum_closed_form(L, anti):
    """Unit links: eigenvalues of m^2 - D_eo D_oe are m^2 + sum_mu sin^2 p_mu.

    Fixes the factor 1/2, the presence and anticommutation of the staggered
    phases, the neighbour offsets per axis and the antiperiodic time momenta
    p_t = (2n+1) pi / L_t.
    """
    m = 0.1
    U = synth.links_unit(L)
    A = H.dense_even_operator(L, lambda f: oracle.apply_A(L, U, m, 0.0, f, anti))
    assert np.max(np.abs(A - A.conj().T)) < 1e-14
    ev = np.linalg.eigvalsh(A)
    ref = H.free_spectrum(L, m, anti)
    assert ev.shape == ref.shape
    assert np.max(np.abs(ev - ref)) < 1e-13


def test_free_field_plane_wave_eigenvectors():
    """Unit links: e^{ip.x} c on even sites is an eigenvector with eigenvalue
    m^2 + sum sin^2 p (antiperiodic time)."""
    L = (4, 6, 4, 8)
    m = 0.3
    U = synth.links_unit(L)
    g = synth.rng(9)
    for _ in range(4):
        n = [g.integers(0, L[mu]) for mu in range(4)]
        p = [2 * np.pi * n[0] / L[0], 2 * np.pi * n[1] / L[1], 2 * np.pi * n[2] / L[2],
             (2 * n[3] + 1) * np.pi / L[3]]
        c = g.standard_normal(3) + 1j * g.standard_normal(3)
        f = H.plane_wave_even(L, p, c)
        lam = m ** 2 + np.sum(np.sin(p) ** 2)
        Af = oracle.apply_A(L, U, m, 0.0, f)
        assert np.max(np.abs(Af - lam * f)) < 1e-13


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 2, 6)])
def test_gauge_covariance(L):
    """D[U^g](g psi) = g D[U] psi with U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag.

    Fixes which link (U(x) forward, U(x-mu)^dag backward) multiplies which
    neighbour, and rules out a transposed link.
    """
    U = synth.links_haar(L, 21)
    g = synth.random_gauge_transform(L, 22)
    psi = synth.gaussian_even_source(L, 1, 23)[0]
    Ug = H.gauge_transform_links(L, U, g)
    lhs = oracle.doe(L, Ug, H.gauge_transform_field(g, psi))
    rhs = H.gauge_transform_field(g, oracle.doe(L, U, psi))
    assert H.max_rel(lhs, rhs) < 1e-14
    chi = synth.gaussian_field(L, 1, 24)[0]
    lhs = oracle.deo(L, Ug, H.gauge_transform_field(g, chi))
    rhs = H.gauge_transform_field(g, oracle.deo(L, U, chi))
    assert H.max_rel(lhs, rhs) < 1e-14


def test_antiperiodic_is_a_time_link_sign():
    """Antiperiodic time equals periodic time with every t-link leaving the
    last time slice negated."""
    L = (2, 4, 2, 4)
    U = synth.links_haar(L, 31)
    psi = synth.gaussian_even_source(L, 1, 32)[0]
    Uflip = U.copy()
    t = synth.site_coords(L)[:, 3]
    Uflip[3, t == L[3] - 1] *= -1
    a = oracle.doe(L, U, psi, antiperiodic=True)
    b = oracle.doe(L, Uflip, psi, antiperiodic=False)
    assert np.max(np.abs(a - b)) < 1e-15


def test_operator_bounds():
    """A = m^2 + D_oe^dag D_oe is Hermitian positive definite with spectrum
    in [m^2 + sigma, m^2 + sigma + 16] (||D|| <= 4: 8 unitary hops of weight 1/2)."""
    L = (4, 4, 4, 4)
    U = synth.links_haar(L, 41)
    m, sig = 0.05, 0.3
    A = H.dense_even_operator(L, lambda f: oracle.apply_A(L, U, m, sig, f))
    assert np.max(np.abs(A - A.conj().T)) < 1e-13
    ev = np.linalg.eigvalsh(A)
    assert ev.min() >= m ** 2 + sig - 1e-12
    assert ev.max() <= m ** 2 + sig + 16 + 1e-12


# ---------------------------------------------------------------- true residual

@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4)])
@pytest.mark.parametrize("sig", [0.0, 0.3])
def test_true_residual_is_dense_relative_two_norm(L, sig):
    """The residual every solver test is judged by (Eq. (2)): ||b - (A + sigma) x||_2
    / ||b||_2 over even sites and colours.  A is assembled densely at sigma = 0
    (the operator is pinned above by its spectrum, covariance and bounds) and
    sigma is added here in numpy, so sigma's handling, the norm (not squared),
    the division by ||b|| and the parity restriction are all checked."""
    m = 0.07
    U = synth.links_haar(L, 61)
    A0 = H.dense_even_operator(L, lambda f: oracle.apply_A(L, U, m, 0.0, f))
    As = A0 + sig * np.eye(A0.shape[0])
    for seed in (62, 63):
        b = synth.gaussian_even_source(L, 1, seed)[0] * 3.7
        x = synth.gaussian_even_source(L, 1, seed + 10)[0] * 0.2
        bv, xv = H.to_even_vector(L, b), H.to_even_vector(L, x)
        ref = np.linalg.norm(bv - As @ xv) / np.linalg.norm(bv)
        got = oracle.true_residual(L, U, m, sig, b, x)
        assert abs(got - ref) <= 1e-14 * ref
        # odd-site entries of the inputs are not part of the even-site vectors
        b2, x2 = b.copy(), x.copy()
        odd = ~H.even_mask(L)
        b2[odd] = 5.0
        x2[odd] = -2.0
        assert abs(oracle.true_residual(L, U, m, sig, b2, x2) - ref) <= 1e-14 * ref
    # near-solution: a dense LAPACK solve leaves a residual at rounding level
    xs = np.linalg.solve(As, bv)
    assert oracle.true_residual(L, U, m, sig, b, H.from_even_vector(L, xs)) <= 1e-13


def test_true_residual_closed_forms():
    """x = 0 gives exactly 1 whatever the scale of b; on the free field a plane
    wave b is an eigenvector (eigenvalue lam = m^2 + sum sin^2 p), so x = c b
    leaves the residual |1 - c (lam + sigma)| exactly."""
    L = (4, 6, 4, 8)
    m, sig = 0.3, 0.25
    U = synth.links_unit(L)
    b = synth.gaussian_even_source(L, 1, 64)[0]
    zero = np.zeros_like(b)
    for scale in (1e-3, 1.0, 42.0):
        assert oracle.true_residual(L, U, m, sig, scale * b, zero) == pytest.approx(1.0, abs=1e-15)
    p = [2 * np.pi / L[0], 0.0, 4 * np.pi / L[2], 3 * np.pi / L[3]]
    f = H.plane_wave_even(L, p, np.array([1.0, 0.5j, -0.25]))
    lam = m ** 2 + np.sum(np.sin(p) ** 2)
    for c in (0.0, 0.5, 1.0 / (lam + sig), 2.0):
        got = oracle.true_residual(L, U, m, sig, f, c * f)
        assert abs(got - abs(1 - c * (lam + sig))) <= 1e-13


# ---------------------------------------------------------------- solvers

@pytest.mark.parametrize("L,gen", [((2, 2, 2, 2), "haar"), ((4, 4, 4, 4), "exp")])
def test_cg_matches_dense_solve(L, gen):
    m, sig = 0.1, 0.0
    U = synth.links_haar(L, 51) if gen == "haar" else synth.links_exp(L, 0.3, 101)
    b = synth.gaussian_even_source(L, 1, 201)[0]
    A = H.dense_even_operator(L, lambda f: oracle.apply_A(L, U, m, sig, f))
    xd = np.linalg.solve(A, H.to_even_vector(L, b))
    x, st, it, tr = oracle.cg(L, U, m, sig, b, tol=1e-12)
    assert st == 0 and tr <= 1e-12
    assert np.max(np.abs(H.to_even_vector(L, x) - xd)) <= 1e-9 * np.max(np.abs(xd))
    assert np.all(x[~H.even_mask(L)] == 0)


def test_cg_free_field_four_eigenvalues():
    """4^4 unit links, antiperiodic: A has exactly four distinct eigenvalues
    (m^2 + 1/2 + {0,1,2,3}), so CG terminates in four steps up to rounding."""
    L = (4, 4, 4, 4)
    m = 0.1
    U = synth.links_unit(L)
    b = synth.gaussian_even_source(L, 1, 202)[0]
    x, st, it, tr = oracle.cg(L, U, m, 0.0, b, tol=1e-10)
    assert st == 0 and tr <= 1e-10
    assert it <= 5
    ev = np.unique(np.round(H.free_spectrum(L, m), 12))
    assert np.allclose(ev, m ** 2 + 0.5 + np.arange(4))


def test_cg_initial_guess_is_used():
    L = (4, 4, 4, 4)
    U = synth.links_exp(L, 0.3, 101)
    b = synth.gaussian_even_source(L, 1, 201)[0]
    x, st, it, tr = oracle.cg(L, U, 0.1, 0.0, b, tol=1e-10)
    x2, st2, it2, tr2 = oracle.cg(L, U, 0.1, 0.0, b, tol=1e-10, x0=x)
    assert st2 == 0 and it2 <= 1


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4)])
def test_multishift_matches_dense_per_shift(L):
    m = 0.02
    U = synth.links_exp(L, 0.5, 103)
    b = synth.gaussian_even_source(L, 1, 203)[0]
    sig = synth.rational_shifts(12)
    X, st, its, tr = oracle.cg_multishift(L, U, m, sig, b, tol=1e-12)
    assert st == 0 and np.all(tr <= 1e-12)
    bv = H.to_even_vector(L, b)
    for k, s in enumerate(sig):
        A = H.dense_even_operator(L, lambda f: oracle.apply_A(L, U, m, s, f))
        xd = np.linalg.solve(A, bv)
        assert np.max(np.abs(H.to_even_vector(L, X[k]) - xd)) <= 1e-9 * np.max(np.abs(xd))


def test_multishift_base_equals_cg_and_needs_no_refinement():
    """The smallest shift follows plain CG exactly (zeta = 1); the shifted
    residuals stay collinear in FP64, so no shift needs refinement."""
    L = (4, 4, 4, 4)
    m = 0.05
    U = synth.links_haar(L, 52)
    b = synth.gaussian_even_source(L, 1, 204)[0]
    sig = np.array([0.5, 0.0, 0.01, 2.0])
    X, st, (it, ref), tr = oracle.cg_multishift(L, U, m, sig, b, tol=1e-10)
    assert st == 0 and ref == 0
    x, st2, it2, tr2 = oracle.cg(L, U, m, 0.0, b, tol=1e-10)
    assert it == it2
    assert np.max(np.abs(X[1] - x)) <= 1e-12 * np.max(np.abs(x))


# ---------------------------------------------------------------- action & force

def _rational_solution(L, U, m, sig, phi, tol=1e-13):
    X = []
    for j in range(phi.shape[0]):
        Xj, st, _, tr = oracle.cg_multishift(L, U, m, sig, phi[j], tol=tol)
        assert st == 0
        X.append(Xj)
    return np.array(X)


def test_action_matches_dense_rational_function():
    """S = sum_j phi_j^dag r(A) phi_j with r(x) = alpha0 + sum_i alpha_i/(x + sigma_i),
    evaluated by dense eigendecomposition."""
    L = (4, 4, 4, 4)
    m = 0.1
    U = synth.links_exp(L, 0.5, 105)
    phi = synth.gaussian_even_source(L, 2, 205)
    sig = synth.rational_shifts(6, 1e-3, 1.0)
    al = synth.rational_weights(sig)
    a0 = 0.3
    X = _rational_solution(L, U, m, sig, phi)
    S = oracle.action(L, a0, al, phi, X)
    A = H.dense_even_operator(L, lambda f: oracle.apply_A(L, U, m, 0.0, f))
    lam, vec = np.linalg.eigh(A)
    r = a0 + sum(a / (lam + s) for a, s in zip(al, sig))
    Sd = 0.0
    for j in range(phi.shape[0]):
        c = vec.conj().T @ H.to_even_vector(L, phi[j])
        Sd += float(np.sum(r * np.abs(c) ** 2))
    assert abs(S - Sd) <= 1e-11 * abs(Sd)


def _action_of(L, U, m, sig, al, phi, tol=1e-13):
    return oracle.action(L, 0.0, al, phi, _rational_solution(L, U, m, sig, phi, tol))


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 2, 4)])
def test_force_vs_central_finite_differences(L):
    """dS/deps along U -> exp(eps T) U equals sum Tr[T F] with F = TA(U M)."""
    m = 0.1
    U = synth.links_exp(L, 0.5, 105)
    phi = synth.gaussian_even_source(L, 2, 205)
    sig = synth.rational_shifts(5, 1e-2, 1.0)
    al = synth.rational_weights(sig)
    X = _rational_solution(L, U, m, sig, phi)
    F = oracle.force(L, U, al, X, mode=0)
    # F is traceless anti-Hermitian
    assert np.max(np.abs(F + np.conj(np.swapaxes(F, -1, -2)))) < 1e-14
    assert np.max(np.abs(np.trace(F, axis1=-2, axis2=-1))) < 1e-14
    T = synth.su3_algebra_directions(L, 4, 305)
    eps = 1e-5
    for d in range(T.shape[0]):
        ana = float(np.real(np.sum(T[d] * np.swapaxes(F, -1, -2))))  # sum Tr[T F]
        Up = H.su3_exp(eps * T[d]) @ U
        Um = H.su3_exp(-eps * T[d]) @ U
        fd = (_action_of(L, Up, m, sig, al, phi) - _action_of(L, Um, m, sig, al, phi)) / (2 * eps)
        assert abs(fd - ana) <= 1e-6 * abs(ana), (d, fd, ana)


def test_force_single_link_directions_exact():
    """On 2^4, for every link and every su(3) generator T, sum Tr[T F] equals
    -2 sum_i alpha_i Re <D_oe X_i, dD_oe X_i>, where dD_oe is the hopping term
    evaluated with the single link U -> T U (the term is real-linear in U)."""
    L = (2, 2, 2, 2)
    V = 16
    m = 0.2
    U = synth.links_haar(L, 61)
    phi = synth.gaussian_even_source(L, 1, 62)
    sig = np.array([0.01, 0.3])
    al = np.array([0.7, 1.3])
    X = _rational_solution(L, U, m, sig, phi)
    F = oracle.force(L, U, al, X, mode=0)
    chi = [oracle.doe(L, U, X[0, i]) for i in range(2)]
    lam = synth._gell_mann()
    worst = 0.0
    for mu in range(4):
        for x in range(V):
            for a in range(8):
                Tm = 1j * lam[a] / 2
                dU = np.zeros_like(U)
                dU[mu, x] = Tm @ U[mu, x]
                ref = sum(-2 * al[i] * np.real(np.vdot(chi[i], oracle.doe(L, dU, X[0, i])))
                          for i in range(2))
                ana = float(np.real(np.trace(Tm @ F[mu, x])))
                worst = max(worst, abs(ref - ana))
    assert worst < 1e-12


def test_raw_force_is_conjugate_wirtinger_gradient():
    """mode 1 returns G = M^dag with dS = Re sum conj(G) dU for any complex dU."""
    L = (2, 4, 2, 2)
    m = 0.2
    U = synth.links_exp(L, 0.4, 71)
    phi = synth.gaussian_even_source(L, 1, 72)
    sig = np.array([0.05, 0.5])
    al = np.array([1.0, 0.5])
    X = _rational_solution(L, U, m, sig, phi)
    G = oracle.force(L, U, al, X, mode=1)
    g = synth.rng(73)
    dU = g.standard_normal(U.shape) + 1j * g.standard_normal(U.shape)
    eps = 1e-6
    fd = (_action_of(L, U + eps * dU, m, sig, al, phi) -
          _action_of(L, U - eps * dU, m, sig, al, phi)) / (2 * eps)
    ana = float(np.real(np.sum(np.conj(G) * dU)))
    assert abs(fd - ana) <= 1e-6 * abs(ana)


def test_force_gauge_covariance():
    """Under (U, phi) -> (U^g, g phi): S is invariant and F_mu(x) -> g(x) F_mu(x) g(x)^dag."""
    L = (4, 4, 2, 2)
    m = 0.1
    U = synth.links_haar(L, 81)
    g = synth.random_gauge_transform(L, 82)
    phi = synth.gaussian_even_source(L, 1, 83)
    sig = np.array([0.01, 0.2])
    al = np.array([1.0, 0.4])
    X = _rational_solution(L, U, m, sig, phi)
    F = oracle.force(L, U, al, X)
    Ug = H.gauge_transform_links(L, U, g)
    phig = H.gauge_transform_field(g, phi[0])[None]
    Xg = _rational_solution(L, Ug, m, sig, phig)
    Fg = oracle.force(L, Ug, al, Xg)
    rot = g[None] @ F @ np.conj(np.swapaxes(g, -1, -2))[None]
    assert H.max_rel(Fg, rot) < 1e-9
    S = oracle.action(L, 0.0, al, phi, X)
    Sg = oracle.action(L, 0.0, al, phig, Xg)
    assert abs(S - Sg) <= 1e-11 * abs(S)
