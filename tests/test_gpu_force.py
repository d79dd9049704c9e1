"""GPU parity of the fermion force and the rational action.

The force kernel is compared with the oracle's force on identical solution
fields X (FP64, <= 1e-12 relative), and the whole chain (GPU solves + GPU
action + GPU force) is checked against central finite differences of the
action along random su(3) directions (eps = 1e-5) and torch's gradcheck.
"""
import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lq():
    import paper_1801_01473_amd as lq
    return lq


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def _pack_many(lq, g, nat):
    return lq.pack_spinor(g, cu(nat.reshape(-1, g.V, 3)), 0)


@pytest.mark.parametrize("L", [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 4), (8, 6, 4, 4)])
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("anti", [True, False])
def test_force_vs_oracle_identical_X(lq, L, mode, anti):
    g = lq.Geometry(L, anti)
    U = synth.links_haar(L, 301)
    npf, ns = 2, 3
    X = synth.gaussian_even_source(L, npf * ns, 302).reshape(npf, ns, -1, 3)
    al = np.array([0.3, 1.1, 2.5])
    U64 = lq.pack_links(g, cu(U))
    F = lq.fermion_force(g, U64, al, _pack_many(lq, g, X), mode=mode)
    got = host(lq.unpack_links(g, F))
    ref = oracle.force(L, U, al, X, mode=mode, antiperiodic=anti)
    assert H.max_rel(got, ref) <= 1e-12


def test_force_accumulate(lq):
    L = (4, 4, 4, 4)
    g = lq.Geometry(L)
    U = synth.links_exp(L, 0.5, 303)
    X = synth.gaussian_even_source(L, 2, 304).reshape(1, 2, -1, 3)
    al = [0.5, 0.25]
    U64 = lq.pack_links(g, cu(U))
    Xp = _pack_many(lq, g, X)
    F1 = lq.fermion_force(g, U64, al, Xp)
    F2 = lq.fermion_force(g, U64, al, Xp, out=F1.clone(), accumulate=True)
    assert (F2 - 2 * F1).abs().max().item() <= 1e-14 * F1.abs().max().item()


def test_action_vs_oracle(lq):
    L = (4, 6, 4, 4)
    g = lq.Geometry(L)
    npf, ns = 3, 4
    phi = synth.gaussian_even_source(L, npf, 305)
    X = synth.gaussian_even_source(L, npf * ns, 306).reshape(npf, ns, -1, 3)
    al = [0.1, 0.2, 0.3, 0.4]
    S = lq.action(g, 0.7, al, _pack_many(lq, g, phi), _pack_many(lq, g, X))
    So = oracle.action(L, 0.7, al, phi, X)
    assert abs(S - So) <= 1e-13 * abs(So)


def _gpu_action(lq, g, U_nat, phi_p, m, sig, al, tol=1e-13):
    U64 = lq.pack_links(g, U_nat if torch.is_tensor(U_nat) else cu(U_nat))
    p = lq.solver_params(mass=m, tol=tol, max_iter=20000)
    X, st, _ = lq.cg_multishift(g, p, U64, sig, phi_p)
    return lq.action(g, 0.0, al, phi_p, X), X, U64


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 4, 2)])
def test_force_vs_finite_differences_16_directions(lq, L):
    """Central differences of S along U -> exp(eps T) U, eps = 1e-5, for 16
    random su(3) directions T, against sum Tr[T F] with F the projected force."""
    g = lq.Geometry(L)
    m = 0.1
    U = synth.links_exp(L, 0.5, 105)
    phi = synth.gaussian_even_source(L, 4, 205)
    phi_p = _pack_many(lq, g, phi)
    sig = synth.rational_shifts(12, 1e-4, 10.0)
    al = synth.rational_weights(sig)
    S0, X, U64 = _gpu_action(lq, g, U, phi_p, m, sig, al)
    Ug = cu(U)
    F = host(lq.unpack_links(g, lq.fermion_force(g, U64, al, X, mode=0)))
    C = synth.su3_algebra_coeffs(L, 16, 305)
    eps = 1e-5
    worst = 0.0
    scale = 0.0
    for d in range(16):
        T = synth.su3_from_coeffs(C[d])
        ana = float(np.real(np.sum(T * np.swapaxes(F, -1, -2))))
        Sp = _gpu_action(lq, g, torch.matmul(cu(synth.expi_coeffs(C[d], eps)), Ug), phi_p, m, sig, al)[0]
        Sm = _gpu_action(lq, g, torch.matmul(cu(synth.expi_coeffs(C[d], -eps)), Ug), phi_p, m, sig, al)[0]
        fd = (Sp - Sm) / (2 * eps)
        worst = max(worst, abs(fd - ana))
        scale = max(scale, abs(ana))
    assert worst <= 1e-6 * scale


def test_fermion_action_gradcheck(lq):
    """torch.autograd.gradcheck of FermionAction on a 2^4 lattice (FP64)."""
    L = (2, 2, 2, 2)
    g = lq.Geometry(L)
    U = cu(synth.links_exp(L, 0.4, 307)).requires_grad_(True)
    phi = _pack_many(lq, g, synth.gaussian_even_source(L, 1, 308))
    sig = [0.05, 0.5]
    al = [1.0, 0.5]
    p = lq.solver_params(mass=0.2, tol=1e-14, max_iter=1000)
    fn = lambda u: lq.FermionAction.apply(u, phi, g, 0.0, al, sig, p)
    assert torch.autograd.gradcheck(fn, (U,), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_force_config5_32(lq):
    """32^4, exp(0.5iH), 12 shifts, 4 pseudofermions: GPU solves to 1e-12,
    then the GPU force equals the oracle force on the same X (all 4 x 12
    (pseudofermion, shift) pairs, both output modes), and its projection
    matches central differences (eps = 1e-5) along 16 random su(3) directions."""
    L = (32, 32, 32, 32)
    g = lq.Geometry(L)
    m = 0.02
    U = synth.links_exp(L, 0.5, 105)
    phi_p = _pack_many(lq, g, synth.gaussian_even_source(L, 4, 205))
    sig = synth.rational_shifts(12)
    al = synth.rational_weights(sig)
    S0, X, U64 = _gpu_action(lq, g, U, phi_p, m, sig, al, tol=1e-12)
    Ug = cu(U)
    F = lq.fermion_force(g, U64, al, X, mode=0)
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(4, 12, -1, 3)
    for mode in (0, 1):
        Fm = F if mode == 0 else lq.fermion_force(g, U64, al, X, mode=1)
        ref = oracle.force(L, U, al, Xn, mode=mode)
        assert H.max_rel(host(lq.unpack_links(g, Fm)), ref) <= 1e-12, mode
        del ref
    del Xn
    Fn = host(lq.unpack_links(g, F))
    C = synth.su3_algebra_coeffs(L, 16, 306)
    eps = 1e-5
    for d in range(C.shape[0]):
        T = synth.su3_from_coeffs(C[d])
        ana = float(np.real(np.sum(T * np.swapaxes(Fn, -1, -2))))
        Sp = _gpu_action(lq, g, torch.matmul(cu(synth.expi_coeffs(C[d], eps)), Ug), phi_p, m, sig, al, 1e-12)[0]
        Sm = _gpu_action(lq, g, torch.matmul(cu(synth.expi_coeffs(C[d], -eps)), Ug), phi_p, m, sig, al, 1e-12)[0]
        fd = (Sp - Sm) / (2 * eps)
        print(f"config 5 direction {d}: fd {fd:.10e} analytic {ana:.10e}", flush=True)
        assert abs(fd - ana) <= 1e-6 * abs(ana), (d, fd, ana)


def test_force_paper_lattice_shape(lq):
    """32^3 x 48 (the paper's lattice, Sec. 5), Haar links, 2 pseudofermions x
    3 shifts solved on the GPU to 1e-12: the projected force and the raw
    gradient equal the oracle's on the same solutions."""
    L = (32, 32, 32, 48)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 4821)
    phi_p = _pack_many(lq, g, synth.gaussian_even_source(L, 2, 4822))
    sig = synth.rational_shifts(3, 1e-2, 1.0)
    al = synth.rational_weights(sig)
    _, X, U64 = _gpu_action(lq, g, U, phi_p, 0.05, sig, al, tol=1e-12)
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(2, 3, -1, 3)
    for mode in (0, 1):
        F = host(lq.unpack_links(g, lq.fermion_force(g, U64, al, X, mode=mode)))
        assert H.max_rel(F, oracle.force(L, U, al, Xn, mode=mode)) <= 1e-12, mode
        del F
