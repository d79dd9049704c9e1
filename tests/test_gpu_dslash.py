"""GPU parity of the packing and D_oe / D_eo kernels against the CPU oracle.

Tolerances (max relative error = max |gpu - oracle| / max |oracle| over all
sites, colours and right-hand sides): FP64 <= 1e-13, FP32 <= 1e-6.
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


SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (4, 2, 6, 4), (6, 4, 2, 8), (8, 8, 8, 8)]


def _links(L, kind, seed):
    if kind == "haar":
        return synth.links_haar(L, seed)
    if kind == "unit":
        return synth.links_unit(L)
    return synth.links_exp(L, 0.5, seed)


@pytest.mark.parametrize("L", SHAPES)
def test_pack_roundtrip(lq, L):
    g = lq.Geometry(L)
    U = synth.links_haar(L, 1)
    Up = lq.pack_links(g, cu(U))
    back = host(lq.unpack_links(g, Up))
    assert np.array_equal(back, U)
    f = synth.gaussian_field(L, 3, 2)
    for par in (0, 1):
        pk = lq.pack_spinor(g, cu(f), par)
        un = host(lq.unpack_spinor(g, pk, par))
        mask = synth.site_parity(L) == par
        assert np.array_equal(un[:, mask], f[:, mask])
        assert np.all(un[:, ~mask] == 0)
    # FP32 rounds to nearest
    pk32 = lq.pack_spinor(g, cu(f), 0, lq.F32)
    un32 = host(lq.unpack_spinor(g, pk32, 0))
    mask = synth.site_parity(L) == 0
    assert np.array_equal(un32[:, mask], f[:, mask].astype(np.complex64).astype(np.complex128))


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (2, 4, 6, 2)])
def test_convert_links_12_reconstructs(lq, L):
    g = lq.Geometry(L)
    U = synth.links_haar(L, 4)
    U64 = lq.pack_links(g, cu(U))
    U12 = lq.convert_links(g, U64, lq.F64, lq.LINKS18, lq.F64, lq.LINKS12)
    back = lq.convert_links(g, U12, lq.F64, lq.LINKS12, lq.F64, lq.LINKS18)
    assert H.max_rel(host(lq.unpack_links(g, back)), U) < 1e-14
    direct12 = lq.pack_links(g, cu(U), lq.F64, lq.LINKS12)
    assert torch.equal(direct12, U12)


@pytest.mark.parametrize("L", SHAPES)
@pytest.mark.parametrize("prec,fmt,tol", [(0, 0, 1e-13), (0, 1, 1e-13), (1, 0, 1e-6), (1, 1, 1e-6)])
@pytest.mark.parametrize("anti", [True, False])
def test_hop_vs_oracle(lq, L, prec, fmt, tol, anti):
    g = lq.Geometry(L, anti)
    U = _links(L, "haar", 10)
    f = synth.gaussian_field(L, 1, 11)[0]
    Up = lq.pack_links(g, cu(U), prec, fmt)
    ev = lq.pack_spinor(g, cu(f[None]), 0, prec)
    od = lq.pack_spinor(g, cu(f[None]), 1, prec)
    got_o = host(lq.unpack_spinor(g, lq.doe(g, Up, ev), 1))[0]
    got_e = host(lq.unpack_spinor(g, lq.deo(g, Up, od), 0))[0]
    ref_o = oracle.doe(L, U, f, anti)
    ref_e = oracle.deo(L, U, f, anti)
    assert H.max_rel(got_o, ref_o) <= tol
    assert H.max_rel(got_e, ref_e) <= tol


@pytest.mark.parametrize("nrhs", [1, 3, 5, 8, 11])
@pytest.mark.parametrize("prec", [0, 1])
def test_multi_rhs_equals_single_rhs(lq, nrhs, prec):
    """Batched right-hand sides give bitwise the single-RHS result per RHS."""
    L = (4, 6, 4, 4)
    g = lq.Geometry(L)
    U = _links(L, "exp", 12)
    fmt = lq.LINKS12 if prec == 1 else lq.LINKS18
    Up = lq.pack_links(g, cu(U), prec, fmt)
    f = synth.gaussian_field(L, nrhs, 13)
    ev = lq.pack_spinor(g, cu(f), 0, prec)
    batched = lq.doe(g, Up, ev)
    for j in range(nrhs):
        single = lq.doe(g, Up, ev[j:j + 1].contiguous())
        assert torch.equal(single[0], batched[j])
    ref = np.stack([oracle.doe(L, U, f[j]) for j in range(nrhs)])
    got = host(lq.unpack_spinor(g, batched, 1))
    assert H.max_rel(got, ref) <= (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("prec,fmt,tol", [(0, 0, 1e-13), (1, 1, 1e-6)])
def test_apply_A_vs_oracle(lq, prec, fmt, tol):
    L = (4, 4, 6, 8)
    g = lq.Geometry(L)
    U = _links(L, "haar", 14)
    b = synth.gaussian_even_source(L, 2, 15)
    Up = lq.pack_links(g, cu(U), prec, fmt)
    x = lq.pack_spinor(g, cu(b), 0, prec)
    got = host(lq.unpack_spinor(g, lq.apply_A(g, Up, 0.1, 0.25, x), 0))
    ref = np.stack([oracle.apply_A(L, U, 0.1, 0.25, b[j]) for j in range(2)])
    assert H.max_rel(got, ref) <= tol


def test_free_field_plane_wave_24(lq):
    """24^4 unit links: even-site plane waves are eigenvectors of A with
    eigenvalue m^2 + sum sin^2 p (closed form, FP64 <= 1e-13)."""
    L = (24, 24, 24, 24)
    g = lq.Geometry(L)
    m = 0.05
    Up = lq.pack_links(g, cu(synth.links_unit(L)))
    r = synth.rng(77)
    for _ in range(2):
        n = r.integers(0, 24, size=4)
        p = 2 * np.pi * n / 24.0
        p[3] = (2 * n[3] + 1) * np.pi / 24.0
        c = r.standard_normal(3) + 1j * r.standard_normal(3)
        f = H.plane_wave_even(L, p, c)
        x = lq.pack_spinor(g, cu(f[None]), 0)
        Ax = lq.apply_A(g, Up, m, 0.0, x)
        lam = m * m + float(np.sum(np.sin(p) ** 2))
        err = (Ax - lam * x).abs().max().item() / x.abs().max().item()
        assert err < 1e-13


def test_anti_hermiticity_gpu(lq):
    L = (8, 8, 8, 8)
    g = lq.Geometry(L)
    U = _links(L, "haar", 16)
    Up = lq.pack_links(g, cu(U))
    f = synth.gaussian_field(L, 2, 17)
    psi = lq.pack_spinor(g, cu(f[0:1]), 0)
    chi = lq.pack_spinor(g, cu(f[1:2]), 1)
    lhs = torch.vdot(chi.flatten(), lq.doe(g, Up, psi).flatten()).item()
    rhs = -torch.vdot(lq.deo(g, Up, chi).flatten(), psi.flatten()).item()
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("prec,fmt,tol", [(0, 0, 1e-13), (1, 1, 1e-6)])
def test_hop_24_vs_oracle(lq, prec, fmt, tol):
    L = (24, 24, 24, 24)
    g = lq.Geometry(L)
    U = _links(L, "haar", 102)
    f = synth.gaussian_even_source(L, 1, 202)[0]
    Up = lq.pack_links(g, cu(U), prec, fmt)
    ev = lq.pack_spinor(g, cu(f[None]), 0, prec)
    got = host(lq.unpack_spinor(g, lq.doe(g, Up, ev), 1))[0]
    assert H.max_rel(got, oracle.doe(L, U, f)) <= tol


@pytest.mark.parametrize("cfg", ["64,1,0,0", "128,2,1,2", "256,4,1,4", "64,8,0,2", "256,8,1,0",
                                 "128,1,1,4", "256,8,1,4,1,0", "128,4,0,2,1,2", "64,2,1,0,0,3",
                                 "256,1,1,2,1,4", "256,1,1,8,0,0,1", "64,2,0,0,1,0,1",
                                 "128,4,1,2,0,2,1", "256,4,1,8,0,0,1,1", "64,2,0,0,0,0,1,1",
                                 "128,8,1,2,0,3,0,1", "256,1,0,0,0,0,0,1",
                                 "256,8,1,0,0,0,0,1,1", "128,4,0,2,0,0,1,0,1",
                                 "64,1,1,8,0,2,0,0,1", "128,2,1,4,1,0,0,1,0,2",
                                 "64,8,0,2,1,0,1,0,1,2", "256,4,1,4,0,3,1,1,1,2",
                                 "128,4,1,2,1,0,0,0,1,2,1", "64,8,0,0,1,3,1,1,0,0,1",
                                 "256,2,1,4,1,0,0,0,0,0,1"])
@pytest.mark.parametrize("prec,fmt,tol", [(0, 0, 1e-13), (1, 1, 1e-6)])
def test_every_launch_configuration(lq, cfg, prec, fmt, tol, monkeypatch):
    """Each (workgroup, RHS block, XCD remap, z-slab or (y, z)-tile traversal,
    non-temporal links, occupancy cap, RHS interleave, loads-first schedule, one
    hop per iteration, non-temporal own-site streams) variant the tuner may pick
    gives the oracle's result;
    ragged RHS count and a lattice whose site count is not a multiple of the
    workgroup."""
    monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
    L = (6, 4, 8, 6)
    g = lq.Geometry(L)
    U = _links(L, "haar", 18)
    f = synth.gaussian_field(L, 5, 19)
    Up = lq.pack_links(g, cu(U), prec, fmt)
    got = host(lq.unpack_spinor(g, lq.doe(g, Up, lq.pack_spinor(g, cu(f), 0, prec)), 1))
    ref = np.stack([oracle.doe(L, U, f[j]) for j in range(5)])
    assert H.max_rel(got, ref) <= tol
    got = host(lq.unpack_spinor(g, lq.deo(g, Up, lq.pack_spinor(g, cu(f), 1, prec)), 0))
    ref = np.stack([oracle.deo(L, U, f[j]) for j in range(5)])
    assert H.max_rel(got, ref) <= tol


@pytest.mark.parametrize("cfg", ["256,8,1,6,1,0,0,0,0,0,1", "256,8,1,6,1,0,0,0,0,6,1",
                                 "128,8,1,6,1,0,0,1,0,4,1", "256,8,1,6,1,0,0,0,1,3,1",
                                 "64,4,0,6,0,0,1,0,0,2,0", "256,8,1,6,1,2,0,0,0,12,1",
                                 "128,2,1,6,1,0,1,0,1,12,1"])
@pytest.mark.parametrize("prec,fmt,tol", [(0, 1, 1e-13), (1, 1, 1e-6)])
def test_six_slice_tiles(lq, cfg, prec, fmt, tol, monkeypatch):
    """(y, z) tiles of six z slices (the tile the tuner picks on 48^4) with
    every row count that divides Ly, each schedule, RHS block 8 over 7
    right-hand sides, on a lattice whose site count is not a multiple of the
    workgroup: D_oe and D_eo against the oracle."""
    monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
    L = (6, 12, 12, 6)
    g = lq.Geometry(L)
    U = _links(L, "haar", 61)
    f = synth.gaussian_field(L, 7, 62)
    Up = lq.pack_links(g, cu(U), prec, fmt)
    fr = f.astype(np.complex64).astype(np.complex128) if prec == 1 else f
    got = host(lq.unpack_spinor(g, lq.doe(g, Up, lq.pack_spinor(g, cu(f), 0, prec)), 1))
    ref = np.stack([oracle.doe(L, U, fr[j]) for j in range(7)])
    assert H.max_rel(got, ref) <= tol
    got = host(lq.unpack_spinor(g, lq.deo(g, Up, lq.pack_spinor(g, cu(f), 1, prec)), 0))
    ref = np.stack([oracle.deo(L, U, fr[j]) for j in range(7)])
    assert H.max_rel(got, ref) <= tol


TM_CFGS = ["64,8,1,0,1,0,0,0,0,0,1,4,4", "128,8,0,0,1,0,0,0,0,0,1,6,2",
           "256,8,1,0,1,0,0,0,0,0,1,12,2", "128,8,1,0,1,2,0,0,0,0,1,4,4",
           "256,8,0,0,1,0,0,0,0,0,1,6,4", "64,8,1,0,1,0,0,0,0,0,1,12,2"]


@pytest.mark.parametrize("cfg", TM_CFGS)
@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 1e-6)])
@pytest.mark.parametrize("nrhs", [8, 11])
def test_t_march_configurations(lq, cfg, prec, tol, nrhs, monkeypatch):
    """The t-march kernel (each thread walks a column along t; 2 or 4 lanes
    share a column's eight right-hand sides) for chunk lengths 4, 6 and 12 of
    Lt = 12, every workgroup size, both XCD maps and an occupancy cap, on
    8 and 11 right-hand sides (a ragged second group): D_oe, D_eo and
    A = m^2 + sigma - D_eo D_oe against the oracle, and bit for bit equal to a
    k_dslash configuration."""
    L = (6, 4, 8, 12)
    g = lq.Geometry(L)
    U = _links(L, "haar", 71)
    f = synth.gaussian_field(L, nrhs, 72)
    fe = f.copy()
    fe[:, synth.site_parity(L) == 1, :] = 0.0
    Up = lq.pack_links(g, cu(U), prec, lq.LINKS12)
    fr = f.astype(np.complex64).astype(np.complex128) if prec == 1 else f
    fer = fe.astype(np.complex64).astype(np.complex128) if prec == 1 else fe
    outs = {}
    for name, c in (("tm", cfg), ("ref", "64,8,1,0,1,0,0,0,0,0,1")):
        monkeypatch.setenv("LQCD_DSLASH_CFG", c)
        outs[name] = (lq.doe(g, Up, lq.pack_spinor(g, cu(f), 0, prec)),
                      lq.deo(g, Up, lq.pack_spinor(g, cu(f), 1, prec)),
                      lq.apply_A(g, Up, 0.1, 0.3, lq.pack_spinor(g, cu(f), 0, prec)))
    for a, b in zip(outs["tm"], outs["ref"]):
        assert torch.equal(a, b)
    got = host(lq.unpack_spinor(g, outs["tm"][0], 1))
    ref = np.stack([oracle.doe(L, U, fr[j]) for j in range(nrhs)])
    assert H.max_rel(got, ref) <= tol
    got = host(lq.unpack_spinor(g, outs["tm"][1], 0))
    ref = np.stack([oracle.deo(L, U, fr[j]) for j in range(nrhs)])
    assert H.max_rel(got, ref) <= tol
    got = host(lq.unpack_spinor(g, outs["tm"][2], 0))
    ref = np.stack([oracle.apply_A(L, U, 0.1, 0.3, fer[j]) for j in range(nrhs)])
    assert H.max_rel(got, ref) <= tol


@pytest.mark.parametrize("cfg", ["256,8,1,0,1,0,0,0,0,0,1,0,2,1", "128,8,0,6,1,0,0,0,0,0,1,0,2,1",
                                 "64,8,1,2,1,0,0,0,0,4,1,0,2,1"])
@pytest.mark.parametrize("nrhs", [8, 11])
def test_matrix_core_stencil(lq, cfg, nrhs, monkeypatch):
    """The matrix-core contraction (one quad of lanes per site, the hop as a
    real 6x6 by 6x8 product on 4x4x1 MFMA blocks), FP32 12-real, eight
    right-hand sides per group (11: a ragged second group), plain and tiled
    traversals, a lattice whose site count is not a multiple of the
    workgroup's sites: D_oe and D_eo against the oracle."""
    monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
    L = (6, 4, 12, 6)
    g = lq.Geometry(L)
    U = _links(L, "haar", 75)
    f = synth.gaussian_field(L, nrhs, 76)
    Up = lq.pack_links(g, cu(U), lq.F32, lq.LINKS12)
    fr = f.astype(np.complex64).astype(np.complex128)
    got = host(lq.unpack_spinor(g, lq.doe(g, Up, lq.pack_spinor(g, cu(f), 0, lq.F32)), 1))
    ref = np.stack([oracle.doe(L, U, fr[j]) for j in range(nrhs)])
    assert H.max_rel(got, ref) <= 1e-6
    got = host(lq.unpack_spinor(g, lq.deo(g, Up, lq.pack_spinor(g, cu(f), 1, lq.F32)), 0))
    ref = np.stack([oracle.deo(L, U, fr[j]) for j in range(nrhs)])
    assert H.max_rel(got, ref) <= 1e-6


def test_t_march_invalid_configuration_falls_back(lq, monkeypatch):
    """A t-march chunk that does not divide Lt is not launched: the call runs
    k_dslash with the remaining settings and still gives the oracle's result."""
    L = (4, 4, 4, 6)
    g = lq.Geometry(L)
    U = _links(L, "haar", 73)
    f = synth.gaussian_field(L, 8, 74)
    Up = lq.pack_links(g, cu(U), lq.F64, lq.LINKS12)
    monkeypatch.setenv("LQCD_DSLASH_CFG", "64,8,1,0,1,0,0,0,0,0,1,4,2")
    got = host(lq.unpack_spinor(g, lq.doe(g, Up, lq.pack_spinor(g, cu(f), 0)), 1))
    ref = np.stack([oracle.doe(L, U, f[j]) for j in range(8)])
    assert H.max_rel(got, ref) <= 1e-13


def test_tuning_cache_file(lq, tmp_path, monkeypatch):
    """LQCD_TUNE_CACHE: a tuned shape is appended to the file; a valid entry
    for the key is used without tuning again (and, every launch variant
    rounding alike, gives the same bits); an invalid entry is ignored and the
    shape is tuned again."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("LQCD_TUNE_CACHE", str(path))
    monkeypatch.delenv("LQCD_DSLASH_CFG", raising=False)
    L = (6, 4, 8, 6)
    g = lq.Geometry(L)
    Up = lq.pack_links(g, cu(_links(L, "haar", 31)))
    x = lq.pack_spinor(g, cu(synth.gaussian_field(L, 1, 32)), 0)
    lq.finalize()
    y1 = lq.doe(g, Up, x)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].count(";") == 1
    key = lines[0].split(";")[0]
    assert key.startswith("v1/") and "/6x4x8x6/" in key
    path.write_text(f"{key};64,1,0,2,0,0,0,0,1,2\n")
    lq.finalize()
    y2 = lq.doe(g, Up, x)
    assert path.read_text().splitlines() == [f"{key};64,1,0,2,0,0,0,0,1,2"]
    assert torch.equal(y1, y2)
    path.write_text(f"{key};96,3,0,5,0,0,0,0,1,2\n")
    lq.finalize()
    y3 = lq.doe(g, Up, x)
    assert len(path.read_text().splitlines()) == 2
    assert torch.equal(y1, y3)
    lq.finalize()


def test_paper_lattice_shape_every_format_8rhs(lq):
    """The paper's lattice shape 32^3 x 48 (Sec. 5; time the longest axis,
    antiperiodic), Haar links, 8 right-hand sides with the tuned launch: D_oe
    and D_eo in the FP64 and FP32 18-real and 12-real formats against the
    oracle on every output site of every right-hand side."""
    L = (32, 32, 32, 48)
    g = lq.Geometry(L)
    U = synth.links_haar(L, 4801)
    fe = synth.gaussian_even_source(L, 8, 4802)
    fo = synth.gaussian_field(L, 8, 4803)
    fo[:, synth.site_parity(L) == 0, :] = 0.0
    ref_oe = np.stack([oracle.doe(L, U, fe[j]) for j in range(8)])
    ref_eo = np.stack([oracle.deo(L, U, fo[j]) for j in range(8)])
    U64 = lq.pack_links(g, cu(U))
    del U
    for prec, fmt, tol in ((lq.F64, lq.LINKS18, 1e-13), (lq.F64, lq.LINKS12, 1e-13),
                           (lq.F32, lq.LINKS18, 1e-6), (lq.F32, lq.LINKS12, 1e-6)):
        Ul = U64 if (prec, fmt) == (lq.F64, lq.LINKS18) else lq.convert_links(
            g, U64, lq.F64, lq.LINKS18, prec, fmt)
        got = host(lq.unpack_spinor(g, lq.doe(g, Ul, lq.pack_spinor(g, cu(fe), 0, prec)), 1))
        assert H.max_rel(got, ref_oe) <= tol, ("D_oe", prec, fmt)
        got = host(lq.unpack_spinor(g, lq.deo(g, Ul, lq.pack_spinor(g, cu(fo), 1, prec)), 0))
        assert H.max_rel(got, ref_eo) <= tol, ("D_eo", prec, fmt)
        del Ul, got


def test_largest_accepted_lattice(lq):
    """The largest lattice class the library accepts (144 Vh just below 2^32,
    here 88^3 x 86, 98 % of the 32-bit offset range of an FP64 18-real link
    block): D_oe and D_eo in FP64 18-real and D_oe in FP32 18-real against
    the oracle on the whole field, with Gaussian 3x3 links (no SU(3) property
    is needed by the 18-real format)."""
    L = (88, 88, 88, 86)
    g = lq.Geometry(L)
    assert 144 * g.Vh < 2 ** 32 and 144 * (88 ** 4 // 2) >= 2 ** 32
    gen = torch.Generator(device="cuda").manual_seed(881)
    Un = torch.randn(4, g.V, 3, 3, dtype=torch.complex128, device="cuda", generator=gen)
    U64 = lq.pack_links(g, Un)
    U = host(Un)
    del Un
    f = host(torch.randn(1, g.V, 3, dtype=torch.complex128, device="cuda", generator=gen))
    threads = oracle.get_threads()
    oracle.set_threads(16)
    try:
        got = host(lq.unpack_spinor(g, lq.doe(g, U64, lq.pack_spinor(g, cu(f), 0)), 1))[0]
        assert H.max_rel(got, oracle.doe(L, U, f[0])) <= 1e-13
        got = host(lq.unpack_spinor(g, lq.deo(g, U64, lq.pack_spinor(g, cu(f), 1)), 0))[0]
        assert H.max_rel(got, oracle.deo(L, U, f[0])) <= 1e-13
        U32 = lq.convert_links(g, U64, lq.F64, lq.LINKS18, lq.F32, lq.LINKS18)
        del U64
        Ur = U.astype(np.complex64).astype(np.complex128)
        fr = f.astype(np.complex64).astype(np.complex128)
        got = host(lq.unpack_spinor(g, lq.doe(g, U32, lq.pack_spinor(g, cu(f), 0, lq.F32)), 1))[0]
        assert H.max_rel(got, oracle.doe(L, Ur, fr[0])) <= 1e-6
    finally:
        oracle.set_threads(threads)
        torch.cuda.empty_cache()


def test_largest_accepted_lattice_8rhs(lq):
    """Eight right-hand sides through one link load at the largest lattice
    class the library accepts (88^3 x 86): FP32 18-real D_oe against the
    oracle for every right-hand side, Gaussian 3x3 links."""
    L = (88, 88, 88, 86)
    g = lq.Geometry(L)
    gen = torch.Generator(device="cuda").manual_seed(882)
    Un = torch.randn(4, g.V, 3, 3, dtype=torch.complex128, device="cuda", generator=gen)
    U32 = lq.pack_links(g, Un, lq.F32, lq.LINKS18)
    Ur = host(Un.to(torch.complex64).to(torch.complex128))
    del Un
    f = torch.randn(8, g.V, 3, dtype=torch.complex128, device="cuda", generator=gen)
    out = lq.doe(g, U32, lq.pack_spinor(g, f, 0, lq.F32))
    del U32
    fr = host(f.to(torch.complex64).to(torch.complex128))
    del f
    threads = oracle.get_threads()
    oracle.set_threads(16)
    try:
        for j in range(8):
            got = host(lq.unpack_spinor(g, out[j:j + 1].contiguous(), 1))[0]
            assert H.max_rel(got, oracle.doe(L, Ur, fr[j])) <= 1e-6, j
    finally:
        oracle.set_threads(threads)
        torch.cuda.empty_cache()
