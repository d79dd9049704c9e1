"""GPU parity of the gauge part of the MD and of whole trajectories.

Gauge action, gauge force, the momentum and link steps and the kinetic
energy against the oracle on identical inputs; a pure-gauge leapfrog
trajectory against the same scheme composed from the oracle's steps;
properties of whole trajectories that hold at any size: reversibility
(integrate, flip the momenta, integrate again: back to the start) and
second-order energy conservation of the Omelyan scheme, for pure gauge and
for RHMC with the fermion force."""
import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

C1 = -1.0 / 12.0


@pytest.fixture(scope="module")
def lq():
    import paper_1801_01473_amd as lq
    return lq


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


LATS = [(4, 4, 4, 4), (2, 2, 2, 2), (4, 2, 6, 4), (6, 4, 4, 8)]


@pytest.mark.parametrize("L", LATS)
@pytest.mark.parametrize("c1", [C1, 0.0])
@pytest.mark.parametrize("method", ["staples", "direct"])
def test_gauge_action_and_force_vs_oracle(lq, L, c1, method):
    """Action and force against the oracle's loop enumeration, for the force
    through staple fields and the direct per-link staple sum, on lattices
    with extents 2 (loops wrapping onto themselves), Symanzik and Wilson."""
    g = lq.Geometry(L)
    U = synth.links_exp(L, 0.7, 501)
    U64 = lq.pack_links(g, cu(U))
    beta = 3.7
    S = lq.gauge_action(g, U64, beta, c1)
    Sref = oracle.gauge_action(L, U, beta, c1)
    assert abs(S - Sref) <= 1e-12 * abs(Sref)
    F = host(lq.unpack_links(g, lq.gauge_force(g, U64, beta, c1, method=method)))
    assert H.max_rel(F, oracle.gauge_force(L, U, beta, c1)) <= 1e-12


@pytest.mark.parametrize("method", ["staples", "direct"])
def test_gauge_force_accumulates(lq, method):
    L = (4, 4, 4, 4)
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, cu(synth.links_haar(L, 502)))
    F1 = lq.gauge_force(g, U64, 2.0, method=method)
    F2 = lq.gauge_force(g, U64, 2.0, out=F1.clone(), accumulate=True, method=method)
    assert (F2 - 2 * F1).abs().max().item() <= 1e-14 * F1.abs().max().item()


def test_gauge_force_methods_agree_at_workload_size(lq):
    """48^4 (the workload lattice), links exp(0.5 i H): the force through
    staple fields equals the direct staple sum on every link (both are
    checked against the oracle on the small lattices above)."""
    L = (48, 48, 48, 48)
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, cu(synth.links_exp(L, 0.5, 519)))
    Fd = lq.gauge_force(g, U64, 5.0, method="direct")
    Fs = lq.gauge_force(g, U64, 5.0, method="staples")
    assert ((Fs - Fd).abs().max() / Fd.abs().max()).item() <= 1e-13


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 2, 6)])
def test_md_steps_and_kinetic_energy_vs_oracle(lq, L):
    g = lq.Geometry(L)
    U = synth.links_haar(L, 503)
    Hn = synth.momenta(L, 504)
    Fn = oracle.gauge_force(L, U, 4.0)
    U64, Hp, Fp = lq.pack_links(g, cu(U)), lq.pack_links(g, cu(Hn)), lq.pack_links(g, cu(Fn))
    assert abs(lq.kinetic_energy(g, Hp) - oracle.kinetic_energy(Hn)) <= 1e-13 * oracle.kinetic_energy(Hn)
    lq.md_update_momenta(g, Hp, Fp, 0.13)
    Hn2 = oracle.md_momenta(Hn, Fn, 0.13)
    assert H.max_rel(host(lq.unpack_links(g, Hp)), Hn2) <= 1e-15
    for eps in (0.05, 0.9):  # 0.9: several squarings in the exponential
        U2 = lq.md_update_links(g, U64.clone(), Hp, eps)
        got = host(lq.unpack_links(g, U2))
        assert H.max_rel(got, oracle.md_links(U, Hn2, eps)) <= 1e-13
        I = np.eye(3)
        assert np.abs(got @ np.conj(np.swapaxes(got, -1, -2)) - I).max() <= 1e-14
        assert np.abs(np.linalg.det(got) - 1).max() <= 1e-14


def _oracle_leapfrog(L, U, Hm, beta, eps, nsteps):
    Hm = oracle.md_momenta(Hm, oracle.gauge_force(L, U, beta), eps / 2)
    for n in range(nsteps):
        U = oracle.md_links(U, Hm, eps)
        Hm = oracle.md_momenta(Hm, oracle.gauge_force(L, U, beta),
                               eps if n < nsteps - 1 else eps / 2)
    return U, Hm


def test_pure_gauge_leapfrog_matches_oracle(lq):
    L = (4, 4, 4, 4)
    g = lq.Geometry(L)
    U = synth.links_exp(L, 0.5, 505)
    Hn = synth.momenta(L, 506)
    beta = 5.0
    U64, Hp = lq.pack_links(g, cu(U)), lq.pack_links(g, cu(Hn))
    lq.md_integrate(g, U64, Hp, 0.2, 4, lambda Ux, F: lq.gauge_force(g, Ux, beta, out=F),
                    integrator="leapfrog")
    Uo, Ho = _oracle_leapfrog(L, U, Hn, beta, 0.05, 4)
    assert H.max_rel(host(lq.unpack_links(g, U64)), Uo) <= 1e-11
    assert H.max_rel(host(lq.unpack_links(g, Hp)), Ho) <= 1e-11


def _energy(lq, g, U64, Hp, beta):
    return lq.kinetic_energy(g, Hp) + lq.gauge_action(g, U64, beta)


@pytest.mark.parametrize("L", [(8, 8, 8, 8), (16, 16, 16, 16)])
def test_pure_gauge_omelyan_reversible_and_second_order(lq, L):
    g = lq.Geometry(L)
    beta = 2.0
    U0 = lq.pack_links(g, cu(synth.links_exp(L, 0.4, 507)))
    H0 = lq.pack_links(g, cu(synth.momenta(L, 508)))
    E0 = _energy(lq, g, U0, H0, beta)
    force = lambda Ux, F: lq.gauge_force(g, Ux, beta, out=F)
    dE = []
    for n in (10, 20):
        U, Hp = U0.clone(), H0.clone()
        lq.md_integrate(g, U, Hp, 0.5, n, force)
        dE.append(_energy(lq, g, U, Hp, beta) - E0)
        if n == 20:  # reversibility: flip the momenta and integrate back
            Hp.neg_()
            lq.md_integrate(g, U, Hp, 0.5, n, force)
            assert (U - U0).abs().max().item() <= 1e-11
            assert (Hp + H0).abs().max().item() <= 1e-10
    assert abs(dE[1]) <= 1e-3 * E0
    assert 3.0 < dE[0] / dE[1] < 5.0


def test_rhmc_trajectory_reversible_and_conserving(lq):
    """With the fermion force (multi-shift solves at tol 1e-12, FP64), the
    trajectory is reversible to the solver tolerance and dH falls with the
    step size as eps^2; the accept decision follows min(1, exp(-dH))."""
    L = (8, 8, 8, 8)
    g = lq.Geometry(L)
    beta, m = 2.0, 0.1
    lo, hi = lq.spectral_bounds(m)
    e8 = lq.minimax(0.125, lo, hi, 10)
    q4 = lq.minimax(-0.25, lo, hi, 10)
    p = lq.solver_params(mass=m, tol=1e-12)
    U0 = lq.pack_links(g, cu(synth.links_exp(L, 0.3, 509)))
    H0 = lq.pack_links(g, cu(synth.momenta(L, 510)))
    xi = lq.pack_spinor(g, cu(synth.gaussian_even_source(L, 1, 511)), 0)
    dH = []
    for n in (8, 16):
        U, Hp = U0.clone(), H0.clone()
        r = lq.rhmc_trajectory(g, p, U, beta, e8, q4, xi, Hp, u=0.0, tau=0.5, nsteps=n)
        # u = 0 accepts every finite dH: the links keep the evolved values
        assert np.isfinite(r["dH"]) and r["accepted"]
        assert (U - U0).abs().max().item() > 1e-3
        assert r["force_evaluations"] == 2 * n + 1
        dH.append(r["dH"])
    assert 2.5 < dH[0] / dH[1] < 6.0  # O(eps^2)
    # reversibility of the MD part with the same pseudofermion field
    phi, _ = lq.pseudofermion_heatbath(g, p, U0, e8, xi)

    def force(Ux, F):
        X, _, _ = lq.cg_multishift(g, p, Ux, q4.sigma, phi)
        lq.fermion_force(g, Ux, q4.alpha, X, out=F)
        lq.gauge_force(g, Ux, beta, out=F, accumulate=True)

    U, Hp = U0.clone(), H0.clone()
    lq.md_integrate(g, U, Hp, 0.5, 4, force)
    Hp.neg_()
    lq.md_integrate(g, U, Hp, 0.5, 4, force)
    assert (U - U0).abs().max().item() <= 1e-9


def test_rhmc_trajectory_reject_restores_links(lq):
    """A coarse trajectory (one Omelyan step over tau = 1) raises H, and with
    u just below 1 the accept/reject step rejects it (exp(-dH) < u): the links
    come back bit for bit.  A finer trajectory (16 steps, dH = O(10), so that
    exp(-dH) > 0) with u = 0 is accepted and leaves the evolved links."""
    L = (8, 8, 8, 8)
    g = lq.Geometry(L)
    beta, m = 2.0, 0.1
    lo, hi = lq.spectral_bounds(m)
    e8 = lq.minimax(0.125, lo, hi, 10)
    q4 = lq.minimax(-0.25, lo, hi, 10)
    p = lq.solver_params(mass=m, tol=1e-12)
    U0 = lq.pack_links(g, cu(synth.links_exp(L, 0.3, 516)))
    H0 = lq.pack_links(g, cu(synth.momenta(L, 517)))
    xi = lq.pack_spinor(g, cu(synth.gaussian_even_source(L, 1, 518)), 0)
    u_hi = float(np.nextafter(1.0, 0.0))
    U, Hp = U0.clone(), H0.clone()
    r = lq.rhmc_trajectory(g, p, U, beta, e8, q4, xi, Hp, u=u_hi, tau=1.0, nsteps=1)
    assert r["dH"] > 1e-6, r["dH"]
    assert not r["accepted"]
    assert torch.equal(U, U0)
    U, Hp = U0.clone(), H0.clone()
    r2 = lq.rhmc_trajectory(g, p, U, beta, e8, q4, xi, Hp, u=0.0, tau=1.0, nsteps=16)
    assert abs(r2["dH"]) < 100.0 < r["dH"], (r2["dH"], r["dH"])
    assert r2["accepted"]
    assert not torch.equal(U, U0)


def test_gauge_force_is_derivative_at_workload_size(lq):
    """48^4 (the workload lattice): dS_g/deps along U -> exp(eps T) U on 16
    scattered links equals sum Tr[T F] there (a property at any size; the
    action and force both from the GPU, the perturbation applied in place)."""
    L = (48, 48, 48, 48)
    g = lq.Geometry(L)
    beta = 5.0
    U64 = lq.pack_links(g, cu(synth.links_exp(L, 0.5, 511)))
    F = lq.gauge_force(g, U64, beta)
    rng = np.random.default_rng(512)
    picks = [(int(rng.integers(2)), int(rng.integers(4)), int(rng.integers(g.Vh))) for _ in range(16)]
    T = torch.from_numpy(synth.su3_from_coeffs(rng.standard_normal((16, 8)))).to("cuda")
    U0 = [U64[p, m, :, h].clone() for p, m, h in picks]
    pred = sum(float(torch.real(torch.trace(T[k] @ F[p, m, :, h].reshape(3, 3))).item())
               for k, (p, m, h) in enumerate(picks))
    eps = 1e-3
    S = []
    for sgn in (1.0, -1.0):
        for k, (p, m, h) in enumerate(picks):
            E = torch.linalg.matrix_exp(sgn * eps * T[k])
            U64[p, m, :, h] = (E @ U0[k].reshape(3, 3)).reshape(9)
        S.append(lq.gauge_action(g, U64, beta))
    d = (S[0] - S[1]) / (2 * eps)
    assert abs(d - pred) <= 1e-5 * max(1.0, abs(pred)), (d, pred)


def test_nested_integrator_reversible_and_second_order(lq):
    """Multi-step integration (fermion force outside, gauge force on 4
    substeps inside): reversible, dH falls as eps^2 in the outer step, and the
    fermion force is evaluated only on the outer level."""
    L = (8, 8, 8, 8)
    g = lq.Geometry(L)
    beta, m = 2.0, 0.1
    lo, hi = lq.spectral_bounds(m)
    e8 = lq.minimax(0.125, lo, hi, 10)
    q4 = lq.minimax(-0.25, lo, hi, 10)
    p = lq.solver_params(mass=m, tol=1e-12)
    U0 = lq.pack_links(g, cu(synth.links_exp(L, 0.3, 513)))
    H0 = lq.pack_links(g, cu(synth.momenta(L, 514)))
    xi = lq.pack_spinor(g, cu(synth.gaussian_even_source(L, 1, 515)), 0)
    dH = []
    for n in (6, 12):
        U, Hp = U0.clone(), H0.clone()
        r = lq.rhmc_trajectory(g, p, U, beta, e8, q4, xi, Hp, u=0.0, tau=0.5, nsteps=n,
                               gauge_substeps=4)
        assert r["force_evaluations"] == 2 * n + 1
        dH.append(r["dH"])
    assert 2.5 < dH[0] / dH[1] < 6.0
    phi, _ = lq.pseudofermion_heatbath(g, p, U0, e8, xi)

    def ferm(Ux, F):
        X, _, _ = lq.cg_multishift(g, p, Ux, q4.sigma, phi)
        lq.fermion_force(g, Ux, q4.alpha, X, out=F)

    gauge = lambda Ux, F: lq.gauge_force(g, Ux, beta, out=F)
    U, Hp = U0.clone(), H0.clone()
    counts = lq.md_integrate_nested(g, U, Hp, 0.5, [3, 4], [ferm, gauge])
    assert counts == [7, 3 * 2 * 9]
    Hp.neg_()
    lq.md_integrate_nested(g, U, Hp, 0.5, [3, 4], [ferm, gauge])
    assert (U - U0).abs().max().item() <= 1e-9
