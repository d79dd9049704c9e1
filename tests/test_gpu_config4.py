"""The batched workload at full size, judged by the oracle system by system.

48^4 Haar links (seed 104), m = 0.02, the 12 rational shifts in [1e-4, 10],
8 Gaussian right-hand sides (seed 204), solved as the benchmark solves them:
mixed precision (FP32 12-real inner iteration, FP64 opening phase, reliable
updates every 100 iterations), right-hand sides batched through each link
load, hipGraph replay, tuned launches (the tuned configurations are printed).
The oracle recomputes the FP64 true residual of all 96 (right-hand side,
shift) systems of Eq. (2); each must be at most 1e-10.  The FP32 12-real
8-RHS D_oe and A = m^2 - D_eo D_oe at this size, with the tuner's launch, are
compared with the oracle on every site of every right-hand side.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

L = (48, 48, 48, 48)
MASS = 0.02


@pytest.fixture(scope="module")
def lq():
    import paper_1801_01473_amd as lq
    return lq


@pytest.fixture(scope="module")
def inputs():
    U = synth.links_haar(L, 104)
    phi = synth.gaussian_even_source(L, 8, 204)
    return U, phi


def _cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _tuned(path):
    return open(path).read() if os.path.exists(path) else "(no tuning cache written)"


def test_config4_every_system_true_residual(lq, inputs, tmp_path, monkeypatch):
    U, phi = inputs
    cache = str(tmp_path / "tune.txt")
    monkeypatch.setenv("LQCD_TUNE_CACHE", cache)
    monkeypatch.delenv("LQCD_DSLASH_CFG", raising=False)
    lq.finalize()
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, _cu(U))
    phi_p = lq.pack_spinor(g, _cu(phi), 0)
    sig = synth.rational_shifts(12)
    p = lq.solver_params(mass=MASS, tol=1e-10, inner_prec=lq.F32, inner_fmt=lq.LINKS12,
                         reliable_interval=100, use_graph=1)
    X, _, stats = lq.cg_multishift(g, p, U64, sig, phi_p)
    print("tuned launches of the solve:\n" + _tuned(cache), flush=True)
    assert all(s["converged"] == 1 for row in stats for s in row)
    worst = 0.0
    for j in range(8):
        xs = lq.unpack_spinor(g, X[j].contiguous(), 0).cpu().numpy()
        for s in range(12):
            tr = oracle.true_residual(L, U, MASS, sig[s], phi[j], xs[s])
            assert tr <= 1e-10, (j, s, tr)
            worst = max(worst, tr)
        del xs
    print(f"largest oracle true residual over 96 systems: {worst:.3e}", flush=True)
    lq.finalize()


def test_config4_fp32_12real_8rhs_stencil(lq, inputs, tmp_path, monkeypatch):
    U, phi = inputs
    cache = str(tmp_path / "tune.txt")
    monkeypatch.setenv("LQCD_TUNE_CACHE", cache)
    monkeypatch.delenv("LQCD_DSLASH_CFG", raising=False)
    lq.finalize()
    g = lq.Geometry(L)
    U64 = lq.pack_links(g, _cu(U))
    U32 = lq.convert_links(g, U64, lq.F64, lq.LINKS18, lq.F32, lq.LINKS12)
    del U64
    x = lq.pack_spinor(g, _cu(phi), 0, lq.F32)
    got = lq.unpack_spinor(g, lq.doe(g, U32, x), 1).cpu().numpy()
    # the oracle sees the FP32-rounded input, so the bar measures the stencil
    phi32 = phi.astype(np.complex64).astype(np.complex128)
    worst = 0.0
    for j in range(8):
        worst = max(worst, H.max_rel(got[j], oracle.doe(L, U, phi32[j])))
    del got
    print("tuned D_oe launch:\n" + _tuned(cache), flush=True)
    assert worst <= 1e-6, worst
    sigma = 0.3
    got = lq.unpack_spinor(g, lq.apply_A(g, U32, MASS, sigma, x), 0).cpu().numpy()
    worst = 0.0
    for j in range(8):
        worst = max(worst, H.max_rel(got[j], oracle.apply_A(L, U, MASS, sigma, phi32[j])))
    print("tuned launches incl. A:\n" + _tuned(cache), flush=True)
    assert worst <= 1e-6, worst
    lq.finalize()
