"""The action entry point that allocates nothing (its block partials sit in the
library's fixed device array) against the workspace entry point, through the C
ABI: the same kernels in the same order, so the results agree bit for bit, on
two calls in a row (the second on a smaller lattice, so the array keeps the
first call's larger contents), plus the oracle's action as a sanity bar."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


def _case(lq, L, npf, nshift, seed):
    g = lq.Geometry(L)
    dev = torch.device("cuda:0")
    phi_nat = synth.gaussian_even_source(L, npf, seed)
    X_nat = synth.gaussian_even_source(L, npf * nshift, seed + 1)
    phi = lq.pack_spinor(g, torch.from_numpy(phi_nat).to(dev), 0)
    X = lq.pack_spinor(g, torch.from_numpy(X_nat).to(dev), 0)
    alpha = [0.1 * (i + 1) for i in range(nshift)]
    return g, phi, X, alpha, phi_nat, X_nat


@pytest.mark.parametrize("order", ["large_then_small"])
def test_action_noalloc_matches_workspace_entry(order):
    import paper_1801_01473_amd as lq

    torch.cuda.set_device(0)
    cases = [((8, 8, 8, 16), 3, 5, 700), ((4, 4, 4, 6), 2, 3, 710)]
    for L, npf, nshift, seed in cases:
        g, phi, X, alpha, phi_nat, X_nat = _case(lq, L, npf, nshift, seed)
        alpha0 = 0.25
        print(f"noalloc action: L={L} npf={npf} nshift={nshift} seed={seed}", flush=True)
        ref = lq.action(g, alpha0, alpha, phi, X)
        got = lq.action_noalloc(g, alpha0, alpha, phi, X)
        assert got == ref, (L, got, ref)
        # and against the oracle's rational action on the same vectors
        Xo = X_nat.reshape(npf, nshift, -1, 3)
        orc = oracle.action(L, alpha0, alpha, phi_nat, Xo)
        assert abs(got - orc) <= 1e-13 * abs(orc), (got, orc)
