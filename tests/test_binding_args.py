"""The binding checks every tensor before calling the library (CPU, no GPU).

Each call below would hand the library a buffer of the wrong precision, size
or layout -- e.g. FP64 links with complex64 spinors, which would make a
stencil read past every row and store FP64 values into a complex64 output.
The binding must raise ValueError naming the argument instead, before any
device work: the tensors are host tensors, so the only check that may fire
last is the one for the device.
"""
import pytest

torch = pytest.importorskip("torch")

import paper_1801_01473_amd as lq  # noqa: E402

G = lq.Geometry((4, 4, 4, 4))
VH = G.Vh


def links(prec=lq.F64, fmt=lq.LINKS18):
    return lq.empty_links(G, prec, fmt, device="cpu")


def spin(n=1, prec=lq.F64):
    return lq.empty_spinor(G, n, prec, device="cpu")


def raises(match, fn, *a, **k):
    with pytest.raises(ValueError, match=match):
        fn(*a, **k)


def test_stencil_precision_mismatch():
    raises("psi_even must be torch.complex128", lq.doe, G, links(), spin(1, lq.F32))
    raises("psi_odd must be torch.complex64", lq.deo, G, links(lq.F32, lq.LINKS12), spin())
    raises("x_even must be torch.complex128", lq.apply_A, G, links(), 0.1, 0.0, spin(1, lq.F32))
    raises("out must be torch.complex128", lq.doe, G, links(), spin(),
           out=spin(1, lq.F32))


def test_stencil_sizes():
    raises("whole number of packed spinors",
           lq.doe, G, links(), torch.zeros(3 * VH + 1, dtype=torch.complex128))
    raises("whole number of packed spinors",
           lq.doe, G, links(), torch.zeros(0, dtype=torch.complex128))
    raises("out must hold 2 packed spinors", lq.doe, G, links(), spin(2), out=spin(1))
    raises("tmp must hold 2 packed spinors", lq.apply_A, G, links(), 0.1, 0.0, spin(2),
           tmp=spin(1))
    raises("packed links", lq.doe, G, torch.zeros(2, 4, 8, VH, dtype=torch.complex128), spin())
    raises("packed links", lq.doe, G, torch.zeros(2, 4, 9, VH + 2, dtype=torch.complex128),
           spin())
    raises("complex128 or complex64", lq.doe, G, torch.zeros(2, 4, 9, VH), spin())


def test_non_contiguous_and_host_tensors():
    s = torch.zeros(1, VH, 3, dtype=torch.complex128).transpose(1, 2)
    raises("psi_even must be contiguous", lq.doe, G, links(), s)
    # everything right but the device: the last check
    raises("must live on the GPU", lq.doe, G, links(), spin())


def test_solvers():
    p = lq.solver_params(mass=0.1)
    raises("b must be torch.complex128", lq.cg, G, p, links(), spin(1, lq.F32))
    raises("x must hold 2 packed spinors", lq.cg, G, p, links(), spin(2), x=spin(1))
    raises("U64 must be torch.complex128", lq.cg, G, p, links(lq.F32), spin())
    raises("U64 must have 9 elements", lq.cg, G, p, links(lq.F64, lq.LINKS12), spin())
    raises("x must hold 6 packed spinors", lq.cg_multishift, G, p, links(), [0.0, 0.1, 0.2],
           spin(2), x=spin(5))
    pm = lq.solver_params(mass=0.1, inner_prec=lq.F32, inner_fmt=lq.LINKS12)
    raises("Uinner must have 6 elements", lq.cg_multishift, G, pm, links(), [0.0], spin(),
           Uinner=links(lq.F32, lq.LINKS18))


def test_force_action_combine():
    al = [0.1, 0.2, 0.3]
    raises("X must be torch.complex128", lq.fermion_force, G, links(), al, spin(3, lq.F32))
    raises("X must hold npf x 3", lq.fermion_force, G, links(), al, spin(4))
    raises("out must be torch.complex128", lq.fermion_force, G, links(), al, spin(3),
           out=links(lq.F32))
    raises("out must have 9 elements", lq.fermion_force, G, links(), al, spin(3),
           out=links(lq.F64, lq.LINKS12))
    raises("X must hold 6 packed spinors", lq.action, G, 0.0, al, spin(2), spin(3))
    raises("X must hold 6 packed spinors", lq.rational_combine, G, 0.0, al, spin(2), spin(3))
    raises("out must hold 2 packed spinors", lq.rational_combine, G, 0.0, al, spin(2),
           spin(6), out=spin(1))


def test_packing_and_links():
    raises("U_nat must be complex128", lq.pack_links, G,
           torch.zeros(4, G.V, 3, 3, dtype=torch.complex64))
    raises("out must have 6 elements", lq.pack_links, G,
           torch.zeros(4, G.V, 3, 3, dtype=torch.complex128), lq.F64, lq.LINKS12, out=links())
    raises("src must be torch.complex64", lq.convert_links, G, links(), lq.F32, lq.LINKS18,
           lq.F64, lq.LINKS12)
    raises("U_packed must be torch.complex128", lq.unpack_links, G, links(lq.F32))
    raises("natural fields must be", lq.pack_spinor, G,
           torch.zeros(2, G.V + 1, 3, dtype=torch.complex128), 0)
    raises("out must hold 2 packed spinors", lq.pack_spinor, G,
           torch.zeros(2, G.V, 3, dtype=torch.complex128), 0, out=spin(1))
    raises("out must be complex128", lq.unpack_spinor, G, spin(2), 0,
           out=torch.zeros(1, G.V, 3, dtype=torch.complex128))


def test_gauge_md_and_smearing():
    raises("U64 must be torch.complex128", lq.gauge_action, G, links(lq.F32), 5.0)
    raises("out must have 9 elements", lq.gauge_force, G, links(), 5.0,
           out=links(lq.F64, lq.LINKS12))
    raises("F must be torch.complex128", lq.md_update_momenta, G, links(), links(lq.F32), 0.1)
    raises("H must have 9 elements", lq.md_update_links, G, links(),
           links(lq.F64, lq.LINKS12), 0.1)
    raises("H must be torch.complex128", lq.kinetic_energy, G, links(lq.F32))
    raises("U64 must have 9 elements", lq.stout_smear, G, links(lq.F64, lq.LINKS12), 0.1)
    raises("G_top must be torch.complex128", lq.stout_force, G, [links(), links()], 0.1,
           links(lq.F32))
    raises("theta must be float64", lq.apply_u1_phases, G, links(),
           torch.zeros(4, G.V, dtype=torch.float32))
