"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function that include/lqcd.h declares,
validate arguments on the host before any device work, and size its buffers
as the paper's byte counts say.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqcd.h")


@pytest.fixture(scope="module")
def lq():
    import paper_1801_01473_amd as lq
    return lq


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lqcd_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["lqcd_doe", "lqcd_deo", "lqcd_cg", "lqcd_cg_multishift",
                     "lqcd_fermion_force", "lqcd_action", "lqcd_pack_links"]:
        assert required in names


def test_library_exports_every_declared_symbol(lq):
    lib = ctypes.CDLL(lq.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(lq.EXPORTED)


def test_status_strings(lq):
    assert lq.status_string(0) == "LQCD_OK"
    assert lq.status_string(5) == "LQCD_ERR_NOT_CONVERGED"
    assert lq.status_string(99) == "LQCD_ERR_UNKNOWN"
    assert lq.version() == 10000


def _golden():
    vals = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_byte_counts.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            vals[k] = int(v)
    return vals


def test_buffer_sizes_match_paper_byte_counts(lq):
    gold = _golden()
    L = (4, 6, 8, 10)
    g = lq.Geometry(L)
    Vh = g.Vh
    # one parity of a FP64 spinor: 48 bytes per site
    assert lq.spinor_bytes(g, lq.F64) == gold["spinor_fp64_bytes_per_site"] * Vh
    assert lq.spinor_bytes(g, lq.F32) == 24 * Vh
    # 12-real FP64 links: 4 directions x 12 doubles per site; a thickness-2
    # slice costs 2 x that per unit of surface
    per_site = lq.links_bytes(g, lq.F64, lq.LINKS12) // g.V
    assert 2 * per_site == gold["gauge_12real_fp64_bytes_per_unit_surface_thickness2"]
    assert lq.links_bytes(g, lq.F64, lq.LINKS18) == 4 * 18 * 8 * g.V
    assert lq.links_bytes(g, lq.F32, lq.LINKS12) == 4 * 12 * 4 * g.V
    # rows 0-1 and the determinant: 14 reals; rows 0-1 and the U(1) angle: 13
    assert lq.links_bytes(g, lq.F32, lq.LINKS12D) == 4 * 14 * 4 * g.V
    assert lq.links_bytes(g, lq.F64, lq.LINKS12T) == 4 * 13 * 8 * g.V
    assert lq.empty_links(g, lq.F32, lq.LINKS12T, "cpu").numel() * 8 == lq.links_bytes(
        g, lq.F32, lq.LINKS12T)


@pytest.mark.parametrize("L", [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 4, 1), (4, -2, 4, 4)])
def test_bad_geometry_is_rejected_before_device_work(lq, L):
    g = lq.lqcd_geom()
    for i in range(4):
        g.L[i] = L[i]
    g.antiperiodic_t = 1
    assert lq._fn("lqcd_links_bytes")(ctypes.byref(g), 0, 0) == 0
    st = lq._fn("lqcd_doe")(ctypes.byref(g), 0, 0, ctypes.c_void_p(16), ctypes.c_void_p(32),
                           ctypes.c_void_p(48), 1, None)
    assert st == lq.ERR_INVALID_ARG
    assert "extent" in lq.last_error()


def test_lattice_size_limit(lq):
    """Byte offsets inside one FP64 18-real link block ([9][Vh] x 16 B) are
    32-bit: 144 Vh must stay below 2^32."""
    g = lq.lqcd_geom()
    for i, n in enumerate((96, 96, 96, 96)):  # Vh = 42467328
        g.L[i] = n
    assert lq._fn("lqcd_links_bytes")(ctypes.byref(g), 0, 0) == 0
    st = lq._fn("lqcd_doe")(ctypes.byref(g), 0, 0, ctypes.c_void_p(16), ctypes.c_void_p(32),
                           ctypes.c_void_p(48), 1, None)
    assert st == lq.ERR_INVALID_ARG and "too large" in lq.last_error()
    for i, n in enumerate((64, 64, 64, 112)):  # Vh = 14680064
        g.L[i] = n
    assert lq._fn("lqcd_links_bytes")(ctypes.byref(g), 0, 0) == 2 * 4 * 9 * 16 * 14680064


def test_bad_arguments_are_rejected(lq):
    g = lq.Geometry((4, 4, 4, 4))
    fn = lq._fn("lqcd_doe")
    # NULL and misaligned pointers, bad enums, nrhs out of range
    assert fn(g.c(), 0, 0, None, ctypes.c_void_p(32), ctypes.c_void_p(48), 1, None) == 1
    assert fn(g.c(), 0, 0, ctypes.c_void_p(17), ctypes.c_void_p(32), ctypes.c_void_p(48), 1,
              None) == 1
    assert fn(g.c(), 2, 0, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(48), 1,
              None) == 1
    assert fn(g.c(), 0, 4, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(48), 1,
              None) == 1
    assert fn(g.c(), 0, 0, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(48), 0,
              None) == 1
    assert fn(g.c(), 0, 0, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(48), 65,
              None) == 1
    assert fn(g.c(), 0, 0, ctypes.c_void_p(16), ctypes.c_void_p(32), ctypes.c_void_p(32), 1,
              None) == 1  # in == out


def test_solver_parameter_validation(lq):
    g = lq.Geometry((4, 4, 4, 4))
    p = lq.solver_params(mass=0.1)
    assert lq.solver_workspace_bytes(g, p, 12, 8) > 0
    for bad in [dict(mass=0.0), dict(mass=-1.0), dict(tol=0.0), dict(tol=1.5), dict(max_iter=0),
                dict(inner_prec=3), dict(inner_fmt=5), dict(rhs_block=3), dict(use_graph=2),
                dict(inner_prec=1, reliable_interval=0), dict(max_refine=-1),
                dict(shift_window=0), dict(shift_window=32), dict(inner_tol_factor=0.0),
                dict(inner_tol_factor=1.5)]:
        kw = dict(mass=0.1)
        kw.update(bad)
        q = lq.solver_params(**kw)
        assert lq.solver_workspace_bytes(g, q, 1, 1) == 0, bad
    assert lq.solver_workspace_bytes(g, p, 0, 1) == 0
    assert lq.solver_workspace_bytes(g, p, 33, 1) == 0
    # deferred shift updates keep the window's residuals: W FP64 vectors per
    # right-hand side beyond the per-iteration layout (W = 31 divides poll 62)
    assert p.shift_window == 31
    p1 = lq.solver_params(mass=0.1, shift_window=1)
    vec = 3 * g.Vh * 16
    extra = lq.solver_workspace_bytes(g, p, 12, 8) - lq.solver_workspace_bytes(g, p1, 12, 8)
    assert extra >= 8 * (31 + 1) * vec
    assert lq.solver_workspace_bytes(g, p, 1, 8) == lq.solver_workspace_bytes(g, p1, 1, 8)
    assert lq.solver_workspace_bytes(g, p, 1, 65) == 0
    # a too-small workspace is reported before any device work
    stats = (lq.SolveStats * 1)()
    sig = (ctypes.c_double * 1)(0.0)
    st = lq._fn("lqcd_cg_multishift")(g.c(), ctypes.byref(p), ctypes.c_void_p(256), None, 1, sig,
                                      ctypes.c_void_p(512), ctypes.c_void_p(1024), 1, stats,
                                      ctypes.c_void_p(4096), 16, None)
    assert st == lq.ERR_WORKSPACE
    sig_bad = (ctypes.c_double * 2)(0.0, -1.0)
    st = lq._fn("lqcd_cg_multishift")(g.c(), ctypes.byref(p), ctypes.c_void_p(256), None, 2,
                                      sig_bad, ctypes.c_void_p(512), ctypes.c_void_p(1024), 1,
                                      stats, ctypes.c_void_p(4096), 1 << 40, None)
    assert st == lq.ERR_INVALID_ARG and "sigma" in lq.last_error()


def test_force_and_action_validation(lq):
    g = lq.Geometry((4, 4, 4, 4))
    al = (ctypes.c_double * 2)(1.0, 2.0)
    f = lq._fn("lqcd_fermion_force")
    v = ctypes.c_void_p
    assert f(g.c(), v(256), 1, 2, al, v(512), 2, 0, v(1024), None) == lq.ERR_INVALID_ARG
    assert f(g.c(), v(256), 0, 2, al, v(512), 0, 0, v(1024), None) == lq.ERR_INVALID_ARG
    assert f(g.c(), v(256), 1, 0, al, v(512), 0, 0, v(1024), None) == lq.ERR_INVALID_ARG
    assert f(g.c(), v(256), 1, 2, al, v(512), 0, 0, v(512), None) == lq.ERR_INVALID_ARG
    S = ctypes.c_double(0)
    a = lq._fn("lqcd_action")
    assert a(g.c(), 1, 2, 0.0, al, v(256), v(512), ctypes.byref(S), v(1024), 8,
             None) == lq.ERR_WORKSPACE
    # the entry point without a workspace: same argument checks, nothing launched
    n = lq._fn("lqcd_action_noalloc")
    assert n(g.c(), 0, 2, 0.0, al, v(256), v(512), ctypes.byref(S), None) == lq.ERR_INVALID_ARG
    assert n(g.c(), 1, 0, 0.0, al, v(256), v(512), ctypes.byref(S), None) == lq.ERR_INVALID_ARG
    assert n(g.c(), 1, 2, 0.0, al, None, v(512), ctypes.byref(S), None) == lq.ERR_INVALID_ARG
    assert n(g.c(), 1, 2, 0.0, al, v(256), v(520), ctypes.byref(S), None) == lq.ERR_INVALID_ARG
    assert n(g.c(), 1, 2, float("nan"), al, v(256), v(512), ctypes.byref(S),
             None) == lq.ERR_INVALID_ARG
    assert n(g.c(), 1, 2, 0.0, al, v(256), v(512), None, None) == lq.ERR_INVALID_ARG
    assert "S must be" in lq.last_error()


def test_bench_traffic_record_is_tied_to_the_profiled_sources(tmp_path, monkeypatch):
    """The bench reports the dominant kernel's counter traffic only for the
    kernel class that was profiled, only while the stencil sources hash to the
    profiled ones and only when the tuner chose the profiled configuration;
    the shipped tuning cache holds that configuration."""
    import json
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "dominant_kernel_traffic.json")))
    assert rec["read_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] > 0
    cfg = rec["tuned_configuration"]
    assert bench.measured_traffic("not_the_profiled_kernel", cfg)[0] is None
    assert bench.measured_traffic(rec["kernel_class"], "64,1,1,0,0,0,0,0,0,0,0,0,2")[0] is None
    got, note = bench.measured_traffic(rec["kernel_class"], cfg)
    assert got == rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"], note
    # the configuration is read back from a tuning cache (last entry of the key)
    L = (48, 48, 48, 48)
    shipped = bench.tuned_config(bench.SHIPPED_TUNE_CACHE, L, rec["kernel_class"], 8)
    assert shipped == cfg
    # (the FP32 classes of an even RHS count run on RHS pairs: keys ending in /pairs)
    cache = tmp_path / "tune.txt"
    key = "v1/gfx950:sramecc+:xnack-/256cu/48x48x48x48/p1/f1/n8/b0/m2"
    cache.write_text(f"{key}/pairs;1,2,1,0,0,0,0,0,0,0\n{key}/pairs;{cfg}\n"
                     f"{key};64,8,1,0,0,0,0,0,0,0\n"
                     "v1/gfx950:sramecc+:xnack-/256cu/48x48x48x48/p1/f1/n8/b0/m0/pairs;2,2\n")
    assert bench.rhs_pairs(rec["kernel_class"], 8)
    assert bench.tuned_config(str(cache), L, rec["kernel_class"], 8) == cfg
    assert bench.tuned_config(str(cache), L, rec["kernel_class"], 4) is None
    assert bench.tuned_config(None, L, rec["kernel_class"], 8) is None
    assert not bench.rhs_pairs("dslash_eo_cg_f64_n8", 8) and not bench.rhs_pairs(
        rec["kernel_class"], 1)
    monkeypatch.setenv("LQCD_RHS_PAIRS", "0")
    assert bench.tuned_config(str(cache), L, rec["kernel_class"], 8) == "64,8,1,0,0,0,0,0,0,0"


def test_gauge_phase_stout_and_rational_validation(lq):
    """The entry points of the rational, gauge-MD, U(1)-phase and stout rows
    reject bad arguments on the host, before any device work; every call
    below is invalid in exactly one respect."""
    g = lq.Geometry((4, 4, 4, 4))
    v = ctypes.c_void_p
    nan, inf = float("nan"), float("inf")
    E, W = lq.ERR_INVALID_ARG, lq.ERR_WORKSPACE

    def rejected(name, *args, code=E, msg=None):
        st = lq._fn(name)(*args)
        assert st == code, (name, args, st, lq.last_error())
        if msg is not None:
            assert msg in lq.last_error(), (name, lq.last_error())

    bad = lq.Geometry((4, 4, 3, 4)).c()         # odd extent

    al = (ctypes.c_double * 2)(1.0, 2.0)
    al_nan = (ctypes.c_double * 2)(1.0, nan)
    rc = "lqcd_rational_combine"
    rejected(rc, bad, 1, 2, 0.5, al, v(256), v(512), v(1 << 30), None, msg="L[2]")
    rejected(rc, g.c(), 0, 2, 0.5, al, v(256), v(512), v(1 << 30), None, msg="nrhs")
    rejected(rc, g.c(), 65, 2, 0.5, al, v(256), v(512), v(1 << 30), None, msg="nrhs")
    rejected(rc, g.c(), 1, 0, 0.5, al, v(256), v(512), v(1 << 30), None, msg="nshift")
    rejected(rc, g.c(), 1, 33, 0.5, al, v(256), v(512), v(1 << 30), None, msg="nshift")
    rejected(rc, g.c(), 1, 2, 0.5, None, v(256), v(512), v(1 << 30), None, msg="alpha")
    rejected(rc, g.c(), 1, 2, 0.5, al_nan, v(256), v(512), v(1 << 30), None, msg="alpha[1]")
    rejected(rc, g.c(), 1, 2, inf, al, v(256), v(512), v(1 << 30), None, msg="alpha0")
    rejected(rc, g.c(), 1, 2, 0.5, al, None, v(512), v(1 << 30), None, msg="b")
    rejected(rc, g.c(), 1, 2, 0.5, al, v(256), v(520), v(1 << 30), None, msg="aligned")
    # y inside X's nrhs*nshift vectors of 3*Vh complex doubles
    rejected(rc, g.c(), 1, 2, 0.5, al, v(256), v(4096), v(4096 + 3 * g.Vh * 16), None,
             msg="overlap")

    ph = "lqcd_apply_u1_phases"
    rejected(ph, g.c(), v(256), None, v(1024), None, msg="theta")
    rejected(ph, g.c(), v(256), v(516), v(1024), None, msg="theta")
    rejected(ph, g.c(), None, v(512), v(1024), None, msg="U64")
    rejected(ph, g.c(), v(256), v(512), v(1032), None, msg="aligned")

    sm = "lqcd_stout_smear"
    rejected(sm, g.c(), v(256), nan, v(1024), None, msg="rho")
    rejected(sm, g.c(), v(256), 0.1, v(256), None, msg="alias")
    rejected(sm, g.c(), v(256), 0.1, None, None, msg="out")
    rejected(sm, bad, v(256), 0.1, v(1024), None)

    ws_need = lq._fn("lqcd_stout_workspace_bytes")(g.c())
    assert ws_need == 2 * 8 * 9 * g.Vh * 16
    assert lq._fn("lqcd_stout_workspace_bytes")(bad) == 0
    sf = "lqcd_stout_force"
    rejected(sf, g.c(), v(256), inf, v(512), 0, v(1024), v(2048), ws_need, None, msg="rho")
    rejected(sf, g.c(), v(256), 0.1, v(512), 2, v(1024), v(2048), ws_need, None, msg="mode")
    rejected(sf, g.c(), v(256), 0.1, v(512), 0, v(1024), v(2048), ws_need - 1, None, code=W)
    rejected(sf, g.c(), v(256), 0.1, v(512), 1, v(256), v(2048), ws_need, None, msg="alias")
    rejected(sf, g.c(), v(256), 0.1, v(512), 1, v(512), v(2048), ws_need, None, msg="alias")
    rejected(sf, g.c(), v(256), 0.1, None, 0, v(1024), v(2048), ws_need, None, msg="G_smeared")
    rejected(sf, g.c(), v(256), 0.1, v(512), 0, v(1024), None, ws_need, None, msg="ws")

    gw = lq._fn("lqcd_gauge_workspace_bytes")(g.c())
    assert gw >= (8 * g.Vh // 256 + 1) * 8 and lq._fn("lqcd_gauge_workspace_bytes")(bad) == 0
    S = ctypes.c_double(0)
    ga = "lqcd_gauge_action"
    rejected(ga, g.c(), v(256), nan, -1 / 12, ctypes.byref(S), v(512), gw, None, msg="beta")
    rejected(ga, g.c(), v(256), 5.0, inf, ctypes.byref(S), v(512), gw, None, msg="c1")
    rejected(ga, g.c(), v(256), 5.0, -1 / 12, None, v(512), gw, None, msg="host")
    rejected(ga, g.c(), v(256), 5.0, -1 / 12, ctypes.byref(S), v(512), gw - 1, None, code=W)
    rejected(ga, g.c(), v(256), 5.0, -1 / 12, ctypes.byref(S), None, gw, None, msg="ws")

    gf = "lqcd_gauge_force"
    rejected(gf, g.c(), v(256), 5.0, -1 / 12, 2, v(1024), None, msg="accumulate")
    rejected(gf, g.c(), v(256), 5.0, -1 / 12, 0, v(256), None, msg="alias")
    rejected(gf, g.c(), v(256), inf, 0.0, 0, v(1024), None, msg="beta")
    rejected(gf, g.c(), v(256), 5.0, 0.0, 0, None, None, msg="F")

    rejected("lqcd_md_update_momenta", g.c(), v(256), nan, v(1024), None, msg="eps")
    rejected("lqcd_md_update_momenta", g.c(), v(256), 0.1, v(256), None, msg="alias")
    rejected("lqcd_md_update_momenta", g.c(), None, 0.1, v(1024), None, msg="F")
    rejected("lqcd_md_update_links", g.c(), v(256), inf, v(1024), None, msg="eps")
    rejected("lqcd_md_update_links", g.c(), v(256), 0.1, v(256), None, msg="alias")
    rejected("lqcd_md_update_links", bad, v(256), 0.1, v(1024), None)

    K = ctypes.c_double(0)
    ke = "lqcd_kinetic_energy"
    rejected(ke, g.c(), v(256), None, v(512), gw, None, msg="host")
    rejected(ke, g.c(), v(256), ctypes.byref(K), v(512), gw - 1, None, code=W)
    rejected(ke, g.c(), v(264), ctypes.byref(K), v(512), gw, None, msg="aligned")


def test_pack_stencil_and_cg_validation(lq):
    """Pack/convert/unpack, D_eo, the operator A and the single-shift solver
    reject bad arguments on the host; every call is invalid in one respect."""
    g = lq.Geometry((4, 4, 4, 4))
    v = ctypes.c_void_p
    E, W = lq.ERR_INVALID_ARG, lq.ERR_WORKSPACE
    bad = lq.Geometry((4, 0, 4, 4)).c()

    def rejected(name, *args, code=E, msg=None):
        st = lq._fn(name)(*args)
        assert st == code, (name, args, st, lq.last_error())
        if msg is not None:
            assert msg in lq.last_error(), (name, lq.last_error())

    pl = "lqcd_pack_links"
    rejected(pl, bad, v(256), 0, 0, v(1024), None, msg="L[1]")
    rejected(pl, g.c(), v(256), 2, 0, v(1024), None)
    rejected(pl, g.c(), v(256), 0, 9, v(1024), None)
    rejected(pl, g.c(), None, 0, 0, v(1024), None, msg="U_nat")
    rejected(pl, g.c(), v(256), 0, 0, v(1025), None, msg="aligned")
    gs = "lqcd_gauge_force_staples"
    need = lq._fn("lqcd_gauge_force_staples_workspace_bytes")(g.c())
    assert need == 4 * 2 * 9 * g.Vh * 16
    rejected(gs, g.c(), v(256), 1.0, 0.0, 0, v(1024), v(4096), need - 1, None,
             code=lq.ERR_WORKSPACE)
    rejected(gs, g.c(), v(256), 1.0, 0.0, 2, v(1024), v(4096), need, None)
    rejected(gs, g.c(), v(256), 1.0, 0.0, 0, v(1024), v(1024), need, None, msg="distinct")
    rejected(gs, g.c(), v(256), 1.0, 0.0, 0, v(1024), None, need, None, msg="ws")
    pu = "lqcd_pack_links_u1"
    rejected(pu, g.c(), None, v(512), 1, v(1024), None, msg="U64")
    rejected(pu, g.c(), v(256), None, 1, v(1024), None, msg="theta")
    rejected(pu, g.c(), v(256), v(512), 2, v(1024), None)
    rejected(pu, g.c(), v(256), v(512), 1, v(256), None, msg="alias")
    rejected(pu, bad, v(256), v(512), 1, v(1024), None)
    cl = "lqcd_convert_links"
    rejected(cl, g.c(), v(256), 0, 0, v(256), 1, 1, None, msg="different")
    rejected(cl, g.c(), v(256), 0, 0, v(1024), 1, 7, None)
    rejected(cl, g.c(), v(256), 5, 0, v(1024), 1, 1, None)
    rejected(cl, g.c(), v(256), 0, 0, None, 1, 1, None, msg="dst")
    rejected("lqcd_unpack_links", g.c(), None, v(1024), None, msg="U_packed")
    rejected("lqcd_unpack_links", bad, v(256), v(1024), None)
    for name in ("lqcd_pack_spinor", "lqcd_unpack_spinor"):
        rejected(name, g.c(), 2, 0, v(256), v(1024), 1, None, msg="parity")
        rejected(name, g.c(), 0, 3, v(256), v(1024), 1, None)
        rejected(name, g.c(), 0, 0, v(256), v(1024), 0, None)
        rejected(name, g.c(), 0, 0, v(256), v(1024), 65, None)
        rejected(name, g.c(), 0, 0, v(256), None, 1, None)

    de = "lqcd_deo"
    rejected(de, g.c(), 0, 0, v(256), v(512), v(512), 1, None, msg="alias")
    rejected(de, g.c(), 0, 0, None, v(512), v(1024), 1, None)
    rejected(de, g.c(), 0, 0, v(256), v(512), v(1024), 65, None)
    rejected(de, g.c(), 1, 4, v(256), v(512), v(1024), 1, None)
    rejected(de, bad, 0, 0, v(256), v(512), v(1024), 1, None)

    aa = "lqcd_apply_A"
    ok = (v(256), 0.1, 0.0, v(512), v(1024), v(2048), 1, None)
    rejected(aa, g.c(), 0, 0, v(256), 0.1, 0.0, v(512), v(512), v(2048), 1, None,
             msg="distinct")
    rejected(aa, g.c(), 0, 0, v(256), 0.1, 0.0, v(512), v(1024), v(512), 1, None,
             msg="distinct")
    rejected(aa, g.c(), 0, 0, v(256), float("nan"), 0.0, v(512), v(1024), v(2048), 1, None,
             msg="finite")
    rejected(aa, g.c(), 0, 0, v(256), 0.1, float("nan"), v(512), v(1024), v(2048), 1, None,
             msg="finite")
    rejected(aa, g.c(), 0, 0, v(256), 0.1, 0.0, v(512), v(1024), None, 1, None, msg="tmp_odd")
    rejected(aa, g.c(), 0, 0, *ok[:-2], 0, None)
    rejected(aa, g.c(), 2, 0, *ok)

    p = lq.solver_params(mass=0.1)
    stats = (lq.SolveStats * 1)()
    cg = "lqcd_cg"
    big = 1 << 40
    rejected(cg, g.c(), ctypes.byref(p), v(256), None, -0.5, v(512), v(1024), 1, stats,
             v(4096), big, None, msg="sigma")
    rejected(cg, g.c(), ctypes.byref(p), v(256), None, 0.0, v(512), v(512), 1, stats,
             v(4096), big, None, msg="alias")
    rejected(cg, g.c(), ctypes.byref(p), v(256), None, 0.0, v(512), v(1024), 1, None,
             v(4096), big, None, msg="host")
    rejected(cg, g.c(), ctypes.byref(p), v(256), v(264), 0.0, v(512), v(1024), 1, stats,
             v(4096), big, None, msg="Uinner")
    rejected(cg, g.c(), ctypes.byref(p), v(256), None, 0.0, v(512), v(1024), 1, stats,
             v(4096), 64, None, code=W)
    rejected(cg, g.c(), ctypes.byref(p), v(256), None, 0.0, v(512), v(1024), 1, stats,
             None, big, None, code=W)
    q = lq.solver_params(mass=0.1, tol=2.0)
    rejected(cg, g.c(), ctypes.byref(q), v(256), None, 0.0, v(512), v(1024), 1, stats,
             v(4096), big, None)


def test_bench_algorithmic_bytes_per_site():
    """The roofline's algorithmic bytes per output site of one D_oe: every link
    once, the input spinor once, the output once.  A spinor site is the
    paper's 48 B in FP64 (Sec. 3.1); 12-real links are 6 complex, and the
    12-real + determinant format 7."""
    import bench
    gold = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_byte_counts.txt")):
        if line.strip() and not line.startswith("#"):
            k, val = line.split()
            gold[k] = int(val)
    spin64 = gold["spinor_fp64_bytes_per_site"]
    assert bench.dslash_bytes_per_site(0, 0, 1) == 8 * 18 * 8 + 2 * spin64 == 1248
    assert bench.dslash_bytes_per_site(1, 0, 1) == 624
    assert bench.dslash_bytes_per_site(1, 1, 1) == 432
    assert bench.dslash_bytes_per_site(0, 1, 1) == 8 * 12 * 8 + 2 * spin64
    for B in (1, 2, 4, 8):
        assert bench.dslash_bytes_per_site(1, 1, B) == 384 + 48 * B
        assert bench.dslash_bytes_per_site(1, 2, B) == 8 * 14 * 4 + 48 * B
        assert bench.dslash_bytes_per_site(0, 1, B) == 768 + B * spin64 * 2


def _builder():
    import importlib.util
    path = os.path.join(ROOT, "paper_1801_01473_amd", "build.py")
    spec = importlib.util.spec_from_file_location("_lqcd_build_t", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_build_resource_guard_parses_and_flags():
    """The build's guard reads the compiler's per-kernel resource remarks and
    flags a kernel with scratch memory (a spill to memory) or a dynamic stack;
    register spills kept in registers (zero scratch) pass."""
    b = _builder()
    text = "\n".join([
        "x.hip:1:1: remark: Function Name: k_good [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:1:1: remark:     VGPRs: 128 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:1:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:1:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:1:1: remark:     SGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:1:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark: Function Name: k_spill [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     VGPRs: 512 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     ScratchSize [bytes/lane]: 96 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     SGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:9:1: remark:     VGPRs Spill: 24 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:19:1: remark: Function Name: k_agpr [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:19:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:19:1: remark:     AGPRs: 90 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:19:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:19:1: remark:     Dynamic Stack: False [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:19:1: remark:     VGPRs Spill: 36 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:29:1: remark: Function Name: k_stack [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:29:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]",
        "x.hip:29:1: remark:     Dynamic Stack: True [-Rpass-analysis=kernel-resource-usage]",
    ])
    recs = b.resource_usage(text)
    assert [r["name"] for r in recs] == ["k_good", "k_spill", "k_agpr", "k_stack"]
    assert recs[1]["vgpr_spill"] == "24" and recs[1]["scratch"] == "96"
    assert [r["name"] for r in b.resource_violations(recs)] == ["k_spill", "k_stack"]
    assert "-Rpass-analysis=kernel-resource-usage" in b.DEVICE_FLAGS


def test_built_kernels_use_no_scratch():
    """Every kernel of the last build: no scratch, no spills, no dynamic stack
    (the reports the build writes beside its objects)."""
    import glob
    reports = glob.glob(os.path.join(ROOT, "_build", "lqcd", "*.o.resources.txt"))
    if not reports:
        pytest.skip("no build reports (library not built in this tree)")
    b = _builder()
    n = 0
    for path in reports:
        recs = [dict(kv.split("=", 1) for kv in line.split()) for line in open(path) if line.strip()]
        n += len(recs)
        assert not b.resource_violations(recs), path
    assert n > 100
