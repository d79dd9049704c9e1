"""GPU solver parity: every solution's true residual, recomputed by the CPU
oracle's FP64 operator, must be <= 1e-10 relative, whatever the inner
precision.  Solutions are also compared with the oracle's own solutions."""
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


def setup(lq, L, links, b_seed, nrhs=1):
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, cu(links))
    b_nat = synth.gaussian_even_source(L, nrhs, b_seed)
    b = lq.pack_spinor(g, cu(b_nat), 0)
    return g, U64, b_nat, b


MODES = [dict(inner_prec=0, inner_fmt=0), dict(inner_prec=1, inner_fmt=1),
         dict(inner_prec=1, inner_fmt=0), dict(inner_prec=0, inner_fmt=1)]


@pytest.mark.parametrize("mode", MODES)
def test_cg_config1(lq, mode):
    """4^4, exp(0.3iH) links, m = 0.1, Gaussian source, tol 1e-10."""
    L = (4, 4, 4, 4)
    U = synth.links_exp(L, 0.3, 101)
    g, U64, b_nat, b = setup(lq, L, U, 201)
    p = lq.solver_params(mass=0.1, tol=1e-10, **mode)
    x, st, stats = lq.cg(g, p, U64, b)
    xn = host(lq.unpack_spinor(g, x, 0))[0]
    tr = oracle.true_residual(L, U, 0.1, 0.0, b_nat[0], xn)
    assert tr <= 1e-10
    assert stats[0]["converged"] == 1 and abs(stats[0]["true_rel_residual"] - tr) < 1e-11
    xo, _, _, _ = oracle.cg(L, U, 0.1, 0.0, b_nat[0], tol=1e-12)
    assert H.max_rel(xn, xo) < 1e-7


def test_cg_free_field_converges_in_four_iterations(lq):
    L = (4, 4, 4, 4)
    g, U64, b_nat, b = setup(lq, L, synth.links_unit(L), 202)
    p = lq.solver_params(mass=0.1, tol=1e-10)
    x, st, stats = lq.cg(g, p, U64, b)
    assert stats[0]["iters"] <= 5 and stats[0]["refine_iters"] == 0


@pytest.mark.parametrize("L", [(4, 4, 4, 4), (6, 4, 2, 8), (8, 8, 8, 8)])
@pytest.mark.parametrize("mode", MODES[:2])
@pytest.mark.parametrize("nrhs", [1, 3, 4])
def test_multishift_every_shift_true_residual(lq, L, mode, nrhs):
    m = 0.02
    U = synth.links_exp(L, 0.5, 103)
    g, U64, b_nat, b = setup(lq, L, U, 203, nrhs)
    sig = synth.rational_shifts(12)
    p = lq.solver_params(mass=m, tol=1e-10, **mode)
    X, st, stats = lq.cg_multishift(g, p, U64, sig, b)
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(nrhs, len(sig), -1, 3)
    for j in range(nrhs):
        for s, sg in enumerate(sig):
            tr = oracle.true_residual(L, U, m, sg, b_nat[j], Xn[j, s])
            assert tr <= 1e-10, (j, s, tr)
            assert stats[j][s]["converged"] == 1


def test_multishift_matches_oracle_solutions(lq):
    L = (4, 4, 4, 4)
    m = 0.05
    U = synth.links_haar(L, 104)
    g, U64, b_nat, b = setup(lq, L, U, 204)
    sig = np.array([0.0, 0.01, 0.1, 1.0])
    p = lq.solver_params(mass=m, tol=1e-10)
    X, st, stats = lq.cg_multishift(g, p, U64, sig, b)
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0))
    Xo, _, _, _ = oracle.cg_multishift(L, U, m, sig, b_nat[0], tol=1e-12)
    for s in range(len(sig)):
        assert H.max_rel(Xn[s], Xo[s]) < 1e-7


def test_batched_rhs_match_single_rhs(lq):
    L = (6, 4, 4, 6)
    m = 0.05
    U = synth.links_exp(L, 0.5, 105)
    g, U64, b_nat, b = setup(lq, L, U, 205, 4)
    sig = synth.rational_shifts(6, 1e-3, 1.0)
    p = lq.solver_params(mass=m, tol=1e-10, inner_prec=1, inner_fmt=1)
    Xb, _, _ = lq.cg_multishift(g, p, U64, sig, b)
    for j in range(4):
        Xs, _, _ = lq.cg_multishift(g, p, U64, sig, b[j:j + 1].contiguous())
        d = (Xs[0] - Xb[j]).abs().max().item() / Xs[0].abs().max().item()
        assert d < 1e-6


@pytest.mark.parametrize("mode", MODES[:2])
@pytest.mark.parametrize("cfg", ["128,4,1,2,1,0,0,0,1,2", "64,2,0,0,1,3,1,1,0,0"])
def test_nontemporal_streams_same_bits(lq, mode, cfg, monkeypatch):
    """Marking the stencils' own-site operands and outputs non-temporal is a
    cache hint only: every stencil mode of the solver (D_oe, the fused CG
    update, the FP64 residual) pinned with and without it gives the same bits,
    and every shift meets the tolerance."""
    L = (8, 4, 6, 4)
    U = synth.links_haar(L, 107)
    g, U64, b_nat, b = setup(lq, L, U, 207, 3)
    sig = synth.rational_shifts(5, 1e-3, 1.0)
    p = lq.solver_params(mass=0.05, tol=1e-10, **mode)
    out = []
    for ns in (0, 1):
        monkeypatch.setenv("LQCD_DSLASH_CFG", f"{cfg},{ns}")
        lq.finalize()
        X, _, stats = lq.cg_multishift(g, p, U64, sig, b)
        assert all(s["converged"] == 1 and s["true_rel_residual"] <= 1e-10
                   for row in stats for s in row)
        out.append(X)
    monkeypatch.delenv("LQCD_DSLASH_CFG")
    lq.finalize()
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("fmt", [1, 0])
@pytest.mark.parametrize("switch", [1e-3, 0.0])
@pytest.mark.parametrize("cfg", ["128,8,1,2,1,3,0,1,1,0,1", "256,4,1,2,1,0,0,1,0,2,1",
                                 "64,2,0,0,0,0,1,0,0,0,0"])
def test_rhs_pairs_same_bits(lq, fmt, switch, cfg, monkeypatch):
    """With an even number of right-hand sides the FP32 phase of a mixed
    multi-shift solve keeps the base direction and D_oe's output as
    interleaved pairs (16-byte stencil accesses, a paired base update).  With
    the stencil configuration pinned, the solutions and every deterministic
    statistic are the same bits as with the systems one after the other
    (LQCD_RHS_PAIRS=0): one-hop and two-hop schedules, RHS blocks 8 (pairs
    past the four systems alias the last one), 4 and 2, cached and
    non-temporal streams, 12- and 18-real links, with and without the FP64
    opening phase (the switch to FP32 and the FP32 start both write pairs),
    through reliable updates; every shift meets the oracle's true residual."""
    L = (8, 4, 6, 4)
    U = synth.links_haar(L, 111)
    g, U64, b_nat, b = setup(lq, L, U, 211, 4)
    sig = synth.rational_shifts(5, 1e-3, 1.0)
    p = lq.solver_params(mass=0.05, tol=1e-10, inner_prec=1, inner_fmt=fmt, mixed_switch=switch)
    keys = ("iters", "reliable_updates", "refine_iters", "converged", "true_rel_residual",
            "iters_fp64", "shift_updates_fp64", "shift_updates_fp32")
    monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
    out = []
    for pairs in ("0", "1"):
        monkeypatch.setenv("LQCD_RHS_PAIRS", pairs)
        lq.finalize()
        X, _, stats = lq.cg_multishift(g, p, U64, sig, b)
        out.append((X, [[{k: s[k] for k in keys} for s in row] for row in stats]))
    monkeypatch.delenv("LQCD_RHS_PAIRS")
    monkeypatch.delenv("LQCD_DSLASH_CFG")
    lq.finalize()
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])
    assert all(s["converged"] == 1 for row in out[1][1] for s in row)
    Xn = host(lq.unpack_spinor(g, out[1][0].reshape(-1, 3, g.Vh), 0)).reshape(4, len(sig), -1, 3)
    for j in range(4):
        for s_, sg in enumerate(sig):
            assert oracle.true_residual(L, U, 0.05, sg, b_nat[j], Xn[j, s_]) <= 1e-10


@pytest.mark.parametrize("nrhs", [2, 6])
@pytest.mark.parametrize("cfg", ["128,8,1,2,1,3,0,1,1,0,1", "256,4,1,2,1,0,0,1,0,2,1"])
def test_rhs_pairs_other_counts(lq, nrhs, cfg, monkeypatch):
    """Right-hand-side pairs at 2 and 6 systems: with RHS blocks of 8 and 4 the
    pairs past the last system alias the last pair (loaded, never stored);
    same bits as separate rows, every shift at the oracle's 1e-10."""
    L = (8, 4, 6, 4)
    U = synth.links_haar(L, 113)
    g, U64, b_nat, b = setup(lq, L, U, 213, nrhs)
    sig = synth.rational_shifts(4, 1e-3, 1.0)
    p = lq.solver_params(mass=0.05, tol=1e-10, inner_prec=1, inner_fmt=1)
    monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
    out = []
    for pairs in ("0", "1"):
        monkeypatch.setenv("LQCD_RHS_PAIRS", pairs)
        lq.finalize()
        X, _, stats = lq.cg_multishift(g, p, U64, sig, b)
        out.append((X, [[(s["iters"], s["true_rel_residual"]) for s in row] for row in stats]))
    monkeypatch.delenv("LQCD_RHS_PAIRS")
    monkeypatch.delenv("LQCD_DSLASH_CFG")
    lq.finalize()
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])
    Xn = host(lq.unpack_spinor(g, out[1][0].reshape(-1, 3, g.Vh), 0)).reshape(nrhs, len(sig), -1, 3)
    for j in range(nrhs):
        for s_, sg in enumerate(sig):
            assert oracle.true_residual(L, U, 0.05, sg, b_nat[j], Xn[j, s_]) <= 1e-10


@pytest.mark.parametrize("mode", [dict(inner_prec=0, inner_fmt=1), MODES[1]])
@pytest.mark.parametrize("tm", ["128,8,1,0,1,0,0,0,0,0,1,4,4", "256,8,0,0,1,0,0,0,0,0,1,8,2"])
def test_t_march_solve_same_bits(lq, mode, tm, monkeypatch):
    """The multi-shift solve of 8 right-hand sides with the t-march stencil
    (D_oe and the fused D_eo + CG update on 12-real links; FP64 and mixed):
    the oracle's true residual of every (right-hand side, shift) is at most
    1e-10, and the solutions agree with a k_dslash configuration's to the
    solver tolerance (not bit for bit: the norm partials are grouped by
    workgroup, and the two kernels' workgroups cover different sites)."""
    L = (8, 8, 8, 8)
    U = synth.links_haar(L, 109)
    g, U64, b_nat, b = setup(lq, L, U, 209, 8)
    sig = synth.rational_shifts(4, 1e-3, 1.0)
    p = lq.solver_params(mass=0.05, tol=1e-10, **mode)
    out = []
    for cfg in (tm, "128,8,1,0,1,0,0,0,0,0,1"):
        monkeypatch.setenv("LQCD_DSLASH_CFG", cfg)
        lq.finalize()
        X, _, stats = lq.cg_multishift(g, p, U64, sig, b)
        assert all(s["converged"] == 1 for row in stats for s in row)
        out.append(X)
    monkeypatch.delenv("LQCD_DSLASH_CFG")
    lq.finalize()
    d = (out[0] - out[1]).abs().max().item() / out[1].abs().max().item()
    assert d < 1e-7, d
    Xn = host(lq.unpack_spinor(g, out[0].reshape(-1, 3, g.Vh), 0)).reshape(8, len(sig), -1, 3)
    for j in range(8):
        for s_, sg in enumerate(sig):
            assert oracle.true_residual(L, U, 0.05, sg, b_nat[j], Xn[j, s_]) <= 1e-10


@pytest.mark.parametrize("mode", MODES[:2])
def test_determinism_and_graph_equivalence(lq, mode):
    """Two runs are bitwise equal, with and without hipGraph replay."""
    L = (8, 4, 6, 4)
    U = synth.links_haar(L, 106)
    g, U64, b_nat, b = setup(lq, L, U, 206, 2)
    sig = synth.rational_shifts(5, 1e-3, 1.0)
    p1 = lq.solver_params(mass=0.05, tol=1e-10, rhs_block=2, use_graph=1, **mode)
    p0 = lq.solver_params(mass=0.05, tol=1e-10, rhs_block=2, use_graph=0, **mode)
    X1, _, s1 = lq.cg_multishift(g, p1, U64, sig, b)
    X2, _, s2 = lq.cg_multishift(g, p1, U64, sig, b)
    X3, _, s3 = lq.cg_multishift(g, p0, U64, sig, b)
    assert torch.equal(X1, X2) and torch.equal(X1, X3)
    assert s1[0][0]["iters"] == s3[0][0]["iters"]


def test_not_converged_reports_stats(lq):
    L = (4, 4, 4, 4)
    U = synth.links_haar(L, 107)
    g, U64, b_nat, b = setup(lq, L, U, 207)
    p = lq.solver_params(mass=0.05, tol=1e-10, max_iter=5, max_refine=0)
    x, st, stats = lq.cg(g, p, U64, b, check=False)
    assert st == lq.ERR_NOT_CONVERGED
    assert stats[0]["iters"] == 5 and stats[0]["converged"] == 0
    assert 1e-10 < stats[0]["true_rel_residual"] < 1.0
    assert "true residual" in lq.last_error()


@pytest.mark.parametrize("mode", [MODES[0], MODES[1]])
def test_nan_source_returns_numeric(lq, mode):
    """A NaN in one element of the second of two right-hand sides: the device
    flags stop the solve, no refinement runs, and both solvers return
    LQCD_ERR_NUMERIC with that system reported as not converged."""
    L = (4, 4, 4, 4)
    U = synth.links_haar(L, 108)
    g, U64, b_nat, b = setup(lq, L, U, 208, nrhs=2)
    b[1, 2, 5] = complex(float("nan"), 0.0)
    p = lq.solver_params(mass=0.1, tol=1e-10, **mode)
    x, st, stats = lq.cg(g, p, U64, b, check=False)
    assert st == lq.ERR_NUMERIC, lq.status_string(st)
    assert "non-finite" in lq.last_error()
    assert stats[1]["converged"] == 0 and stats[1]["refine_iters"] == 0
    X, st, stats = lq.cg_multishift(g, p, U64, [0.0, 0.5, 2.0], b, check=False)
    assert st == lq.ERR_NUMERIC, lq.status_string(st)
    assert all(s["converged"] == 0 and s["refine_iters"] == 0 for s in stats[1])
    with pytest.raises(lq.LqcdError) as e:
        lq.cg_multishift(g, p, U64, [0.0, 0.5], b)
    assert e.value.status == lq.ERR_NUMERIC


def test_cg_initial_guess(lq):
    L = (4, 4, 4, 4)
    U = synth.links_exp(L, 0.3, 101)
    g, U64, b_nat, b = setup(lq, L, U, 201)
    p = lq.solver_params(mass=0.1, tol=1e-10)
    x, _, s0 = lq.cg(g, p, U64, b)
    x2, _, s1 = lq.cg(g, p, U64, b, x=x.clone())
    assert s1[0]["iters"] <= 1 and s1[0]["converged"] == 1


def test_zero_source_gives_zero_solution(lq):
    L = (4, 4, 4, 4)
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, cu(synth.links_haar(L, 1)))
    b = torch.zeros((1, 3, g.Vh), dtype=torch.complex128, device="cuda")
    X, st, stats = lq.cg_multishift(g, lq.solver_params(mass=0.1), U64, [0.0, 1.0], b)
    assert st == 0 and X.abs().max().item() == 0.0 and stats[0][0]["iters"] == 0


def test_cg_config2_24(lq):
    """24^4 Haar links, m = 0.05, plain FP64 CG to 1e-10."""
    L = (24, 24, 24, 24)
    U = synth.links_haar(L, 102)
    g, U64, b_nat, b = setup(lq, L, U, 202)
    p = lq.solver_params(mass=0.05, tol=1e-10)
    x, st, stats = lq.cg(g, p, U64, b)
    xn = host(lq.unpack_spinor(g, x, 0))[0]
    assert oracle.true_residual(L, U, 0.05, 0.0, b_nat[0], xn) <= 1e-10


def test_multishift_config3_32_mixed(lq):
    """32^4, exp(0.5iH), m = 0.02, 12 shifts in [1e-4, 10], FP32 12-real inner
    with FP64 reliable updates every 100 iterations: every shift <= 1e-10."""
    L = (32, 32, 32, 32)
    m = 0.02
    U = synth.links_exp(L, 0.5, 103)
    g, U64, b_nat, b = setup(lq, L, U, 203)
    sig = synth.rational_shifts(12)
    p = lq.solver_params(mass=m, tol=1e-10, inner_prec=1, inner_fmt=1, reliable_interval=100)
    X, st, stats = lq.cg_multishift(g, p, U64, sig, b)
    assert st == 0
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0))
    for s, sg in enumerate(sig):
        tr = oracle.true_residual(L, U, m, sg, b_nat[0], Xn[s])
        assert tr <= 1e-10, (s, tr)


def test_phase_counters_and_two_phase_switch(lq):
    """Mixed multi-shift runs an FP64 opening phase then FP32; the counters
    report it consistently, and an FP64 solve reports all its work as FP64."""
    L = (8, 8, 8, 8)
    U = synth.links_exp(L, 0.5, 108)
    g, U64, b_nat, b = setup(lq, L, U, 208, 2)
    sig = synth.rational_shifts(6, 1e-3, 1.0)
    pm = lq.solver_params(mass=0.05, tol=1e-10, inner_prec=1, inner_fmt=1, mixed_switch=1e-3)
    X, st, stats = lq.cg_multishift(g, pm, U64, sig, b)
    for row in stats:
        s0 = row[0]
        assert 0 < s0["iters_fp64"] < s0["iters"]
        assert s0["iters_fp64"] <= s0["shift_updates_fp64"] <= s0["iters_fp64"] * len(sig)
        n32 = s0["iters"] - s0["iters_fp64"]
        assert n32 <= s0["shift_updates_fp32"] <= n32 * len(sig)
    p64 = lq.solver_params(mass=0.05, tol=1e-10)
    X64, st, s64 = lq.cg_multishift(g, p64, U64, sig, b)
    for row in s64:
        assert row[0]["iters_fp64"] == row[0]["iters"] and row[0]["shift_updates_fp32"] == 0
    # both reach the same solutions within the tolerance
    d = (X - X64).abs().max().item() / X64.abs().max().item()
    assert d < 1e-6
    # FP32 throughout (no opening phase) also meets the bar, through refinement
    p0 = lq.solver_params(mass=0.05, tol=1e-10, inner_prec=1, inner_fmt=1, mixed_switch=0.0)
    X0, st, s0 = lq.cg_multishift(g, p0, U64, sig, b)
    Xn = host(lq.unpack_spinor(g, X0.reshape(-1, 3, g.Vh), 0)).reshape(2, len(sig), -1, 3)
    for j in range(2):
        for s, sg in enumerate(sig):
            assert oracle.true_residual(L, U, 0.05, sg, b_nat[j], Xn[j, s]) <= 1e-10
        assert s0[j][0]["iters_fp64"] == 0


def test_stream_bandwidth_reports(lq):
    c, t = lq.stream_bandwidth(1 << 26, 3)
    assert c > 100.0 and t > 100.0


def test_kernel_timing_instrumentation(lq):
    """Timing mode brackets every D_oe, D_eo and shift-update launch of the
    main solve with events; counts match the iteration counts and the
    solution equals the graph-replayed one bitwise."""
    L = (8, 8, 4, 4)
    U = synth.links_exp(L, 0.5, 109)
    g, U64, b_nat, b = setup(lq, L, U, 209, 2)
    sig = synth.rational_shifts(4, 1e-2, 1.0)
    p = lq.solver_params(mass=0.1, tol=1e-10, inner_prec=1, inner_fmt=1)
    Xg, _, sg = lq.cg_multishift(g, p, U64, sig, b)
    lq.kernel_timing(True)
    Xt, _, st = lq.cg_multishift(g, p, U64, sig, b)
    lq.kernel_timing(False)
    kt = lq.kernel_timing()
    assert torch.equal(Xg, Xt)
    # deferred shift updates: K5 forms the base direction, K6 flushes each window
    n64 = kt["base_update_f64_n2"][0]
    n32 = kt["base_update_f32_n2"][0]
    it64 = st[0][0]["iters_fp64"]
    # launches come in blocks of the poll interval, so there can be a few more than iterations
    assert n64 >= it64 and n32 >= st[0][0]["iters"] - it64
    assert kt["dslash_oe_f64_n2"][0] == n64 and kt["dslash_eo_cg_f32_n2"][0] == n32
    w = st[0][0]["shift_window"]
    assert w == 31
    # one scheduled flush per window, plus the forced ones at phase ends and reliable updates
    assert kt["ms_flush_f64_n2"][0] >= n64 // w and kt["ms_flush_f32_n2"][0] >= n32 // w
    assert all(ms > 0 for _, ms in kt.values())
    # the per-iteration shift update is back with shift_window = 1
    p1 = lq.solver_params(mass=0.1, tol=1e-10, inner_prec=1, inner_fmt=1, shift_window=1)
    lq.kernel_timing(True)
    X1, _, s1 = lq.cg_multishift(g, p1, U64, sig, b)
    lq.kernel_timing(False)
    kt1 = lq.kernel_timing()
    assert "ms_update_f32_n2" in kt1 and "ms_flush_f32_n2" not in kt1
    assert s1[0][0]["shift_window"] == 1 and s1[0][0]["flush_slots_fp32"] == 0
    assert (X1 - Xt).abs().max().item() / Xt.abs().max().item() < 1e-6
    lq.kernel_timing(True)
    assert lq.kernel_timing() == {}
    lq.kernel_timing(False)


@pytest.mark.parametrize("mode", MODES[:2])
@pytest.mark.parametrize("window,poll", [(1, 0), (20, 40), (7, 0), (4, 6), (31, 0), (31, 31)])
def test_deferred_shift_updates_match(lq, mode, window, poll):
    """Deferred shift updates (x_s, p_s kept as combinations of the window's
    base residuals, Sec. 2 recurrences regrouped) reach every shift's true
    residual bar for any window length, including ones that are not a divisor
    of the poll interval (reduced to one) and the longest window; every
    iteration's residual is combined by exactly one flush."""
    L = (6, 4, 4, 8)
    m = 0.03
    U = synth.links_haar(L, 110)
    g, U64, b_nat, b = setup(lq, L, U, 210, 2)
    sig = synth.rational_shifts(7, 1e-4, 3.0)
    p = lq.solver_params(mass=m, tol=1e-10, shift_window=window, poll_interval=poll, **mode)
    X, st, stats = lq.cg_multishift(g, p, U64, sig, b)
    assert st == 0
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(2, len(sig), -1, 3)
    pol = poll if poll else (31 if mode["inner_prec"] == 1 else 62)
    w_expect = max(d for d in range(1, min(window, 31) + 1) if pol % d == 0)
    for j in range(2):
        for s, sg in enumerate(sig):
            assert oracle.true_residual(L, U, m, sg, b_nat[j], Xn[j, s]) <= 1e-10, (j, s)
        r = stats[j][0]
        assert r["shift_window"] == w_expect
        if w_expect > 1:
            assert r["flush_slots_fp64"] + r["flush_slots_fp32"] == r["iters"]
            assert r["flush_shifts_fp64"] + r["flush_shifts_fp32"] <= (
                r["shift_updates_fp64"] + r["shift_updates_fp32"])
            assert r["flush_shifts_fp64"] >= r["flush_slots_fp64"] // w_expect
        else:
            assert r["flush_slots_fp64"] == r["flush_slots_fp32"] == 0
    Xo, _, _, _ = oracle.cg_multishift(L, U, m, sig, b_nat[0], tol=1e-12)
    for s in range(len(sig)):
        assert H.max_rel(Xn[0, s], Xo[s]) < 1e-7



def test_inner_tol_factor_margin(lq):
    """A tighter stopping margin makes the main iteration run longer and every
    (rhs, shift) still meets tol; factor 1 stops exactly at tol."""
    L = (8, 8, 8, 8)
    m = 0.03
    U = synth.links_haar(L, 111)
    g, U64, b_nat, b = setup(lq, L, U, 211, 2)
    sig = synth.rational_shifts(6, 1e-4, 1.0)
    its = {}
    for f in (1.0, 0.5):
        p = lq.solver_params(mass=m, tol=1e-10, inner_prec=1, inner_fmt=1, inner_tol_factor=f)
        X, st, stats = lq.cg_multishift(g, p, U64, sig, b)
        assert st == 0
        Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(2, len(sig), -1, 3)
        for j in range(2):
            for s_, sg in enumerate(sig):
                assert oracle.true_residual(L, U, m, sg, b_nat[j], Xn[j, s_]) <= 1e-10
        its[f] = stats[0][0]["iters"]
    assert its[0.5] > its[1.0]


def test_multishift_paper_lattice_shape_mixed(lq):
    """The paper's lattice shape 32^3 x 48, Haar links, m = 0.02, 12 shifts in
    [1e-4, 10], 2 right-hand sides, FP32 12-real inner with FP64 reliable
    updates: every (rhs, shift) <= 1e-10 by the oracle's true residual."""
    L = (32, 32, 32, 48)
    m = 0.02
    U = synth.links_haar(L, 4811)
    g, U64, b_nat, b = setup(lq, L, U, 4812, 2)
    sig = synth.rational_shifts(12)
    p = lq.solver_params(mass=m, tol=1e-10, inner_prec=1, inner_fmt=1, reliable_interval=100)
    X, st, stats = lq.cg_multishift(g, p, U64, sig, b)
    assert st == 0
    Xn = host(lq.unpack_spinor(g, X.reshape(-1, 3, g.Vh), 0)).reshape(2, len(sig), -1, 3)
    for j in range(2):
        for s, sg in enumerate(sig):
            tr = oracle.true_residual(L, U, m, sg, b_nat[j], Xn[j, s])
            assert tr <= 1e-10, (j, s, tr)
