"""GPU parity with U(1) phases on the links (Sec. 4.1): the phase kernel, the
Dirac operator, the multi-shift solver (FP64 and mixed precision with 18-real
inner links) and the fermion force on phased links, against the oracle on the
same phased links."""
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


def _theta(L, kind):
    if kind == "chemical":
        return synth.u1_phases_chemical(L, 0.37)
    if kind == "magnetic":
        return synth.u1_phases_magnetic(L, 2) + synth.u1_phases_chemical(L, -0.2)
    return synth.u1_phases_pure_gauge(L, 801)[0]


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 2, 8), (8, 8, 8, 8)])
@pytest.mark.parametrize("kind", ["chemical", "magnetic", "gauge"])
def test_phased_links_and_dslash(lq, L, kind):
    g = lq.Geometry(L)
    U = synth.links_haar(L, 802)
    th = _theta(L, kind)
    Up_ref = oracle.phase_links(U, th)
    U64 = lq.pack_links(g, cu(U))
    Up = lq.apply_u1_phases(g, U64, cu(th))
    assert H.max_rel(host(lq.unpack_links(g, Up)), Up_ref) <= 1e-15
    # in place gives the same
    U64b = U64.clone()
    lq.apply_u1_phases(g, U64b, cu(th), out=U64b)
    assert torch.equal(U64b, Up)
    f = synth.gaussian_even_source(L, 2, 803)
    ref = np.stack([oracle.doe(L, Up_ref, f[j]) for j in range(2)])
    got = host(lq.unpack_spinor(g, lq.doe(g, Up, lq.pack_spinor(g, cu(f), 0)), 1))
    assert H.max_rel(got, ref) <= 1e-13
    U32 = lq.convert_links(g, Up, lq.F64, lq.LINKS18, lq.F32, lq.LINKS18)
    got32 = host(lq.unpack_spinor(g, lq.doe(g, U32, lq.pack_spinor(g, cu(f), 0, lq.F32)), 1))
    assert H.max_rel(got32, ref) <= 1e-6


@pytest.mark.parametrize("inner", [(0, 0), (1, 0)])
def test_multishift_with_chemical_potential(lq, inner):
    """Every (rhs, shift) meets 1e-10 on the FP64 phased operator (true
    residual recomputed by the oracle); mixed precision with 18-real inner
    links (phased links are not SU(3))."""
    L = (8, 8, 8, 8)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 804)
    th = synth.u1_phases_chemical(L, 0.5) + synth.u1_phases_magnetic(L, 1)
    Up_ref = oracle.phase_links(U, th)
    Up = lq.apply_u1_phases(g, lq.pack_links(g, cu(U)), cu(th))
    b = synth.gaussian_even_source(L, 2, 805)
    sig = synth.rational_shifts(6, 1e-3, 1.0)
    m = 0.05
    p = lq.solver_params(mass=m, tol=1e-10, inner_prec=inner[0], inner_fmt=inner[1])
    X, _, stats = lq.cg_multishift(g, p, Up, sig, lq.pack_spinor(g, cu(b), 0))
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(2, len(sig), -1, 3)
    for j in range(2):
        for i, s in enumerate(sig):
            assert oracle.true_residual(L, Up_ref, m, s, b[j], Xn[j, i]) <= 1e-10
    assert all(s["converged"] == 1 for row in stats for s in row)


def test_fermion_force_on_phased_links(lq):
    L = (4, 4, 4, 4)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 806)
    th = synth.u1_phases_magnetic(L, 1) + synth.u1_phases_chemical(L, 0.8)
    Up_ref = oracle.phase_links(U, th)
    Up = lq.apply_u1_phases(g, lq.pack_links(g, cu(U)), cu(th))
    X = synth.gaussian_even_source(L, 2 * 3, 807).reshape(2, 3, -1, 3)
    al = np.array([0.4, 1.2, 2.0])
    F = lq.fermion_force(g, Up, al, lq.pack_spinor(g, cu(X.reshape(-1, g.V, 3)), 0))
    assert H.max_rel(host(lq.unpack_links(g, F)), oracle.force(L, Up_ref, al, X)) <= 1e-12


def test_links12d_round_trip_and_dslash(lq):
    """The 12-real + determinant format keeps phased (non-SU(3)) links exact:
    pack / convert round trips, D_oe in FP64 and FP32 against the oracle, and
    the SU(3)-only 12-real format is wrong on the same links."""
    L = (6, 4, 4, 8)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 808)
    th = synth.u1_phases_magnetic(L, 3) + synth.u1_phases_chemical(L, 0.45)
    Up_ref = oracle.phase_links(U, th)
    Up = lq.apply_u1_phases(g, lq.pack_links(g, cu(U)), cu(th))
    U12d = lq.pack_links(g, cu(Up_ref), lq.F64, lq.LINKS12D)
    back = lq.convert_links(g, U12d, lq.F64, lq.LINKS12D, lq.F64, lq.LINKS18)
    assert H.max_rel(host(lq.unpack_links(g, back)), Up_ref) <= 1e-14
    c12d = lq.convert_links(g, Up, lq.F64, lq.LINKS18, lq.F64, lq.LINKS12D)
    assert torch.equal(c12d, U12d) or (c12d - U12d).abs().max().item() <= 1e-15
    f = synth.gaussian_even_source(L, 3, 809)
    ref = np.stack([oracle.doe(L, Up_ref, f[j]) for j in range(3)])
    for prec, tol in ((lq.F64, 1e-13), (lq.F32, 1e-6)):
        Ul = lq.convert_links(g, Up, lq.F64, lq.LINKS18, prec, lq.LINKS12D)
        got = host(lq.unpack_spinor(g, lq.doe(g, Ul, lq.pack_spinor(g, cu(f), 0, prec)), 1))
        assert H.max_rel(got, ref) <= tol
    U12 = lq.convert_links(g, Up, lq.F64, lq.LINKS18, lq.F64, lq.LINKS12)
    bad = host(lq.unpack_spinor(g, lq.doe(g, U12, lq.pack_spinor(g, cu(f), 0)), 1))
    assert H.max_rel(bad, ref) > 1e-3


def test_links12t_flavour_angles_and_dslash(lq):
    """The paper's U(1) storage: SU(3) rows 0-1 plus one angle per link, the
    phase recomputed in the operator.  Built per flavour from the shared SU(3)
    field and that flavour's angles, or converted from phased links (angle =
    arg det / 3): round trip to the phased links, D_oe in FP64 and FP32 against
    the oracle on u U, for two flavours with different charges."""
    L = (6, 4, 4, 8)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 816)
    U64 = lq.pack_links(g, cu(U))
    f = synth.gaussian_even_source(L, 3, 817)
    fo = synth.gaussian_field(L, 3, 822)
    fo[:, synth.site_parity(L) == 0, :] = 0.0
    for charge in (1.0, -2.0 / 3.0):
        th = charge * (synth.u1_phases_magnetic(L, 3) + synth.u1_phases_chemical(L, 0.45))
        Up_ref = oracle.phase_links(U, th)
        ref = np.stack([oracle.doe(L, Up_ref, f[j]) for j in range(3)])
        Up = lq.apply_u1_phases(g, U64, cu(th))
        for prec, tol in ((lq.F64, 1e-13), (lq.F32, 1e-6)):
            Ut = lq.pack_links_u1(g, U64, cu(th), prec)
            back = lq.convert_links(g, Ut, prec, lq.LINKS12T, lq.F64, lq.LINKS18)
            assert H.max_rel(host(lq.unpack_links(g, back)), Up_ref) <= (
                1e-14 if prec == lq.F64 else 1e-6)
            got = host(lq.unpack_spinor(g, lq.doe(g, Ut, lq.pack_spinor(g, cu(f), 0, prec)), 1))
            assert H.max_rel(got, ref) <= tol, (charge, prec)
            Uc = lq.convert_links(g, Up, lq.F64, lq.LINKS18, prec, lq.LINKS12T)
            got = host(lq.unpack_spinor(g, lq.deo(g, Uc, lq.pack_spinor(g, cu(fo), 1, prec)), 0))
            ref_eo = np.stack([oracle.deo(L, Up_ref, fo[j]) for j in range(3)])
            assert H.max_rel(got, ref_eo) <= tol, (charge, prec)
        Ub = lq.pack_links(g, cu(Up_ref), lq.F64, lq.LINKS12T)
        assert H.max_rel(host(lq.unpack_links(
            g, lq.convert_links(g, Ub, lq.F64, lq.LINKS12T, lq.F64, lq.LINKS18))), Up_ref) <= 1e-14


@pytest.mark.parametrize("cfg", ["64,1,0,0", "128,2,1,2,1,0,0,1,1,2", "256,8,1,4,1,3,0,0,1,0,1",
                                 "128,4,0,2,1,0,1,0,0,2,1"])
def test_links12t_every_launch_configuration(lq, cfg, monkeypatch):
    monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
    L = (6, 4, 8, 6)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 818)
    th = synth.u1_phases_chemical(L, -0.7) + synth.u1_phases_magnetic(L, 2)
    Up_ref = oracle.phase_links(U, th)
    Ul = lq.pack_links_u1(g, lq.pack_links(g, cu(U)), cu(th), lq.F32)
    f = synth.gaussian_field(L, 5, 819)
    got = host(lq.unpack_spinor(g, lq.deo(g, Ul, lq.pack_spinor(g, cu(f), 1, lq.F32)), 0))
    ref = np.stack([oracle.deo(L, Up_ref, f[j]) for j in range(5)])
    assert H.max_rel(got, ref) <= 1e-6


def test_multishift_phased_links12t_inner(lq):
    """Mixed precision with the angle format as the inner links (converted by
    the solver from the FP64 phased links, also for its FP64 opening phase),
    and with the caller's per-flavour angle links as the inner copy: every
    (rhs, shift) <= 1e-10 by the oracle's true residual."""
    L = (8, 8, 8, 8)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 820)
    th = synth.u1_phases_chemical(L, 0.5) + synth.u1_phases_magnetic(L, 1)
    Up_ref = oracle.phase_links(U, th)
    U64 = lq.pack_links(g, cu(U))
    Up = lq.apply_u1_phases(g, U64, cu(th))
    b = synth.gaussian_even_source(L, 2, 821)
    sig = synth.rational_shifts(6, 1e-3, 1.0)
    m = 0.05
    p = lq.solver_params(mass=m, tol=1e-10, inner_prec=lq.F32, inner_fmt=lq.LINKS12T)
    for Uin in (None, lq.pack_links_u1(g, U64, cu(th), lq.F32)):
        X, _, stats = lq.cg_multishift(g, p, Up, sig, lq.pack_spinor(g, cu(b), 0), Uinner=Uin)
        Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(2, len(sig), -1, 3)
        for j in range(2):
            for i, s in enumerate(sig):
                assert oracle.true_residual(L, Up_ref, m, s, b[j], Xn[j, i]) <= 1e-10
        assert all(s["converged"] == 1 for row in stats for s in row)


@pytest.mark.parametrize("cfg", ["64,1,0,0", "128,2,1,2,1,0,0,1,1,2", "256,8,1,4,1,3,0,0,1,0,1",
                                 "128,4,0,2,1,0,1,0,0,2,1", "64,8,0,0,0,2,0,1,0,0"])
def test_links12d_every_launch_configuration(lq, cfg, monkeypatch):
    monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
    L = (6, 4, 8, 6)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 810)
    th = synth.u1_phases_chemical(L, -0.7)
    Up_ref = oracle.phase_links(U, th)
    Ul = lq.convert_links(g, lq.apply_u1_phases(g, lq.pack_links(g, cu(U)), cu(th)),
                          lq.F64, lq.LINKS18, lq.F32, lq.LINKS12D)
    f = synth.gaussian_field(L, 5, 811)
    got = host(lq.unpack_spinor(g, lq.deo(g, Ul, lq.pack_spinor(g, cu(f), 1, lq.F32)), 0))
    ref = np.stack([oracle.deo(L, Up_ref, f[j]) for j in range(5)])
    assert H.max_rel(got, ref) <= 1e-6


def test_multishift_phased_links12d_inner(lq):
    """Mixed precision with the compressed phased format as the inner links
    (and as the FP64 opening phase's links): every (rhs, shift) <= 1e-10."""
    L = (8, 8, 8, 8)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 812)
    th = synth.u1_phases_chemical(L, 0.5) + synth.u1_phases_magnetic(L, 1)
    Up_ref = oracle.phase_links(U, th)
    Up = lq.apply_u1_phases(g, lq.pack_links(g, cu(U)), cu(th))
    b = synth.gaussian_even_source(L, 2, 813)
    sig = synth.rational_shifts(6, 1e-3, 1.0)
    m = 0.05
    p = lq.solver_params(mass=m, tol=1e-10, inner_prec=lq.F32, inner_fmt=lq.LINKS12D)
    X, _, stats = lq.cg_multishift(g, p, Up, sig, lq.pack_spinor(g, cu(b), 0))
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(2, len(sig), -1, 3)
    for j in range(2):
        for i, s in enumerate(sig):
            assert oracle.true_residual(L, Up_ref, m, s, b[j], Xn[j, i]) <= 1e-10
    assert all(s["converged"] == 1 for row in stats for s in row)


def test_phased_dslash_at_workload_size(lq):
    """48^4 (the workload lattice), magnetic + chemical phases: D_oe on the
    phased links in the 12-real + determinant format (FP64, FP32) and in
    18-real FP64 against the oracle, every output site."""
    L = (48, 48, 48, 48)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 814)
    th = synth.u1_phases_magnetic(L, 5) + synth.u1_phases_chemical(L, 0.3)
    Up = lq.apply_u1_phases(g, lq.pack_links(g, cu(U)), cu(th))
    Up_ref = oracle.phase_links(U, th)
    del U
    f = synth.gaussian_even_source(L, 1, 815)
    ref = oracle.doe(L, Up_ref, f[0])[None]
    del Up_ref
    for prec, fmt, tol in ((lq.F64, lq.LINKS18, 1e-13), (lq.F64, lq.LINKS12D, 1e-13),
                           (lq.F32, lq.LINKS12D, 1e-6), (lq.F64, lq.LINKS12T, 1e-13),
                           (lq.F32, lq.LINKS12T, 1e-6)):
        Ul = Up if (prec, fmt) == (lq.F64, lq.LINKS18) else lq.convert_links(
            g, Up, lq.F64, lq.LINKS18, prec, fmt)
        got = host(lq.unpack_spinor(g, lq.doe(g, Ul, lq.pack_spinor(g, cu(f), 0, prec)), 1))
        assert H.max_rel(got, ref) <= tol, (prec, fmt)
        del Ul
