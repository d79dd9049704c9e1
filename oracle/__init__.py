"""ctypes wrapper of the plain FP64 CPU oracle (``oracle/lqcd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  All
arrays are numpy complex128 in natural lexicographic layout (see the C file).

Parity status: every function here is pinned in ``tests/test_oracle.py``
(closed-form free-field spectrum, anti-Hermiticity, gauge covariance, dense
LAPACK solves, exact derivatives and finite differences; ``true_residual``
against the dense relative 2-norm and closed forms at x = 0 and on a
free-field plane wave); ``rational_apply`` in ``tests/test_rational.py``
(dense eigendecomposition of A); ``stout_smear`` / ``stout_force`` in
``tests/test_stout.py`` (the single-link weak-field closed form, which fixes
the sign and scale of rho, the rise of the plaquette, covariance, finite
differences).  The one convention
those pins cannot fix is the order of the staggered phases over the axes,
eta_mu(x) = (-1)^(x_0 + ... + x_{mu-1}) with (x, y, z, t) = (0, 1, 2, 3):
any ordering gives the same spectrum and symmetries, so that ordering is a
stated convention shared with the GPU path, not a pinned result.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lqcd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblqcd_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_hop.argtypes = [_ip, ctypes.c_int, _dp, _dp, _dp, ctypes.c_int]
    lib.orc_doe.argtypes = [_ip, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_deo.argtypes = [_ip, ctypes.c_int, _dp, _dp, _dp]
    lib.orc_apply_A.argtypes = [_ip, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double,
                                _dp, _dp, _dp]
    lib.orc_true_residual.argtypes = [_ip, ctypes.c_int, _dp, ctypes.c_double,
                                      ctypes.c_double, _dp, _dp]
    lib.orc_true_residual.restype = ctypes.c_double
    lib.orc_cg.argtypes = [_ip, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double, _dp,
                           _dp, ctypes.c_double, ctypes.c_int, _ip, _dp]
    lib.orc_cg.restype = ctypes.c_int
    lib.orc_cg_multishift.argtypes = [_ip, ctypes.c_int, _dp, ctypes.c_double, ctypes.c_int,
                                      _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp,
                                      ctypes.c_int]
    lib.orc_cg_multishift.restype = ctypes.c_int
    lib.orc_action.argtypes = [_ip, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
    lib.orc_action.restype = ctypes.c_double
    lib.orc_force.argtypes = [_ip, ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int, _dp, _dp,
                              ctypes.c_int, _dp]
    lib.orc_gauge_action.argtypes = [_ip, _dp, ctypes.c_double, ctypes.c_double]
    lib.orc_gauge_action.restype = ctypes.c_double
    lib.orc_gauge_force.argtypes = [_ip, _dp, ctypes.c_double, ctypes.c_double, _dp]
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_get_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _geom(L):
    arr = (ctypes.c_int * 4)(*[int(v) for v in L])
    if any(int(v) < 2 or int(v) % 2 for v in L):
        raise ValueError(f"every extent must be even and >= 2, got {tuple(L)}")
    return arr


def _c128(a, shape):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _ptr(a):
    return a.ctypes.data_as(_dp)


def _V(L):
    return int(L[0]) * int(L[1]) * int(L[2]) * int(L[3])


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def hop(L, U, psi, out_parity: int, antiperiodic: bool = True) -> np.ndarray:
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    psi = _c128(psi, (V, 3))
    out = np.zeros((V, 3), np.complex128)
    _load().orc_hop(_geom(L), int(antiperiodic), _ptr(U), _ptr(psi), _ptr(out), int(out_parity))
    return out


def doe(L, U, psi_even, antiperiodic: bool = True) -> np.ndarray:
    """D_oe: even-site input -> odd-site output (natural layout, other parity zero)."""
    return hop(L, U, psi_even, 1, antiperiodic)


def deo(L, U, psi_odd, antiperiodic: bool = True) -> np.ndarray:
    """D_eo: odd-site input -> even-site output."""
    return hop(L, U, psi_odd, 0, antiperiodic)


def apply_A(L, U, mass: float, sigma: float, x, antiperiodic: bool = True) -> np.ndarray:
    """((m^2 + sigma) - D_eo D_oe) x on even sites."""
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    x = _c128(x, (V, 3))
    y = np.zeros((V, 3), np.complex128)
    tmp = np.zeros((V, 3), np.complex128)
    _load().orc_apply_A(_geom(L), int(antiperiodic), _ptr(U), float(mass) ** 2, float(sigma),
                        _ptr(x), _ptr(y), _ptr(tmp))
    return y


def true_residual(L, U, mass, sigma, b, x, antiperiodic: bool = True) -> float:
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    b = _c128(b, (V, 3))
    x = _c128(x, (V, 3))
    return float(_load().orc_true_residual(_geom(L), int(antiperiodic), _ptr(U),
                                           float(mass) ** 2, float(sigma), _ptr(b), _ptr(x)))


def cg(L, U, mass, sigma, b, tol=1e-10, max_iter=10000, x0=None, antiperiodic=True):
    """Returns (x, status, iterations, true relative residual)."""
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    b = _c128(b, (V, 3))
    x = np.zeros((V, 3), np.complex128) if x0 is None else _c128(x0, (V, 3)).copy()
    it = ctypes.c_int(0)
    tr = ctypes.c_double(0.0)
    st = _load().orc_cg(_geom(L), int(antiperiodic), _ptr(U), float(mass) ** 2, float(sigma),
                        _ptr(b), _ptr(x), float(tol), int(max_iter), ctypes.byref(it),
                        ctypes.byref(tr))
    return x, int(st), int(it.value), float(tr.value)


def cg_multishift(L, U, mass, sigmas, b, tol=1e-10, max_iter=10000, antiperiodic=True,
                  verify=True):
    """Returns (x [nshift][V][3], status, (ms_iters, refine_iters), true_res [nshift]).

    verify=False skips the final per-shift residual recomputation and CG
    refinement (true_res is then NaN)."""
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    b = _c128(b, (V, 3))
    sig = np.ascontiguousarray(sigmas, dtype=np.float64)
    ns = sig.size
    x = np.zeros((ns, V, 3), np.complex128)
    iters = (ctypes.c_int * 2)(0, 0)
    tr = np.zeros(ns, np.float64)
    st = _load().orc_cg_multishift(_geom(L), int(antiperiodic), _ptr(U), float(mass) ** 2, ns,
                                   _ptr(sig), _ptr(b), _ptr(x), float(tol), int(max_iter),
                                   iters, _ptr(tr), 1 if verify else 0)
    return x, int(st), (int(iters[0]), int(iters[1])), tr


def gauge_action(L, U, beta: float, c1: float = -1.0 / 12.0) -> float:
    """Tree-level Symanzik gauge action (Sec. 2): beta sum over every 1x1
    plaquette (weight c0 = 1 - 8 c1) and every 1x2 rectangle in both
    orientations (weight c1) of (1 - Re Tr W / 3).  c1 = 0: Wilson."""
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    return float(_load().orc_gauge_action(_geom(L), _ptr(U), float(beta), float(c1)))


def gauge_force(L, U, beta: float, c1: float = -1.0 / 12.0) -> np.ndarray:
    """F = TA(U M), dS_g = sum Re Tr[dU M] (the convention of ``force`` mode 0),
    natural [4][V][3][3]."""
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    F = np.zeros((4, V, 3, 3), np.complex128)
    _load().orc_gauge_force(_geom(L), _ptr(U), float(beta), float(c1), _ptr(F))
    return F


def phase_links(U, theta) -> np.ndarray:
    """u_mu(x) U_mu(x) with u = exp(i theta_mu(x)) (Sec. 4.1: the U(1) field of
    each flavour -- imaginary chemical potential, background fields -- enters
    the Dirac operator as a factor on the links).  U natural [4][V][3][3],
    theta [4][V]; every oracle function then takes the phased links as U."""
    U = np.asarray(U, dtype=np.complex128)
    return U * np.exp(1j * np.asarray(theta, dtype=np.float64))[..., None, None]


def _shift_index(L, mu, d):
    """lex index of x + d mu^ for every x (periodic)."""
    V = _V(L)
    lex = np.arange(V)
    c = [lex % L[0], (lex // L[0]) % L[1], (lex // (L[0] * L[1])) % L[2],
         lex // (L[0] * L[1] * L[2])]
    c[mu] = (c[mu] + d) % L[mu]
    return c[0] + L[0] * (c[1] + L[1] * (c[2] + L[2] * c[3]))


def _dag(A):
    return np.conj(np.swapaxes(A, -1, -2))


def _ta(W):
    Y = 0.5 * (W - _dag(W))
    tr = np.trace(Y, axis1=-2, axis2=-1)[..., None, None]
    return Y - tr / 3.0 * np.eye(3)


def _expm_ah(X):
    """exp(X) for anti-Hermitian X (stack): eigendecomposition of -iX."""
    w, v = np.linalg.eigh(-1j * X)
    return np.einsum("...ij,...j,...kj->...ik", v, np.exp(1j * w), v.conj())


def _stout_parts(L, U, rho, mu):
    """Staple sum A_mu (plaquettes: Tr[U_mu A_mu] is the plaquette), X = TA(rho A^dag U^dag)."""
    A = np.zeros_like(U[mu])
    xp = _shift_index(L, mu, 1)
    for nu in range(4):
        if nu == mu:
            continue
        xn, xm = _shift_index(L, nu, 1), _shift_index(L, nu, -1)
        xpm = xp[xm]
        A += U[nu][xp] @ _dag(U[mu][xn]) @ _dag(U[nu])
        A += _dag(U[nu][xpm]) @ _dag(U[mu][xm]) @ U[nu][xm]
    X = _ta(rho * _dag(A) @ _dag(U[mu]))
    return A, X


def stout_smear(L, U, rho: float) -> np.ndarray:
    """One level of stout smearing (the smeared links U^(k) of the Dirac
    operator, Sec. 2): U' = exp(X) U, X = TA(Omega), Omega = rho C U^dag with
    C = sum over nu != mu of the plaquette staples of the link (isotropic rho).
    Natural [4][V][3][3]."""
    U = np.asarray(U, dtype=np.complex128)
    out = np.empty_like(U)
    for mu in range(4):
        _, X = _stout_parts(L, U, rho, mu)
        out[mu] = _expm_ah(X) @ U[mu]
    return out


def stout_force(L, U, rho: float, G_smeared, mode: int = 0) -> np.ndarray:
    """Chain rule through one smearing level: given the raw gradient with
    respect to the smeared links, G' = M'^dag (dS = sum Re Tr[dU' M']), return
    F = TA(U M) (mode 0) or M^dag (mode 1) with dS = sum Re Tr[dU M], the
    exact derivative written out: U' = E U, E = exp(X):
      Re Tr[M' E dU]                      -> M += M' E
      Re Tr[U M' dE] = Re Tr[L(X, U M') dX], L(X, B) the top-right block of
        exp([[X, B], [0, X]]); with dX = TA(dOmega) this is Re Tr[Lam dOmega],
        Lam = TA(L(X, U M')), and dOmega = rho (dA^dag U^dag + A^dag dU^dag):
        -> M += rho A Lam^dag, and Re Tr[dA K], K = rho Lam^dag U, spread over
        every link of every staple in A (each link of the product in turn)."""
    from scipy.linalg import expm
    U = np.asarray(U, dtype=np.complex128)
    Mp = _dag(np.asarray(G_smeared, dtype=np.complex128))
    M = np.zeros_like(U)
    V = _V(L)
    for mu in range(4):
        A, X = _stout_parts(L, U, rho, mu)
        E = _expm_ah(X)
        B = U[mu] @ Mp[mu]
        G = np.empty_like(B)
        Z = np.zeros((6, 6), np.complex128)
        for x in range(V):
            Z[:3, :3] = X[x]
            Z[3:, 3:] = X[x]
            Z[:3, 3:] = B[x]
            G[x] = expm(Z)[:3, 3:]
        Lam = _ta(G)
        M[mu] += Mp[mu] @ E + rho * A @ _dag(Lam)
        K = rho * _dag(Lam) @ U[mu]
        xp = _shift_index(L, mu, 1)
        for nu in range(4):
            if nu == mu:
                continue
            xn, xm = _shift_index(L, nu, 1), _shift_index(L, nu, -1)
            xpm = xp[xm]
            x = np.arange(V)
            for path in ([(nu, xp, False), (mu, xn, True), (nu, x, True)],
                         [(nu, xpm, True), (mu, xm, True), (nu, xm, False)]):
                mats = [_dag(U[d][i]) if dg else U[d][i] for d, i, dg in path]
                for k in range(3):
                    # R = P_{k+1} ... P_3 K P_1 ... P_{k-1}
                    R = np.broadcast_to(np.eye(3), K.shape).copy()
                    for q in range(k + 1, 3):
                        R = R @ mats[q]
                    R = R @ K
                    for q in range(0, k):
                        R = R @ mats[q]
                    d, i, dg = path[k]
                    np.add.at(M[d], i, _dag(R) if dg else R)
    return _ta(U @ M) if mode == 0 else _dag(M)


def md_momenta(H, F, eps: float) -> np.ndarray:
    """Momentum step of the MD (Sec. 4.3 and Alg. 2, "new momenta"): with U' = i H U and the
    force F = TA(U M) of ``force`` / ``gauge_force`` (dS/deps = sum Tr[T F]
    for U -> exp(eps T) U), energy conservation of H^2/2 + S gives
    H' = -i F, so H <- H - i eps F.  Natural [4][V][3][3]."""
    return np.asarray(H, dtype=np.complex128) - 1j * float(eps) * np.asarray(F)


def md_links(U, H, eps: float) -> np.ndarray:
    """Link step of the MD ("new configuration"): U <- exp(i eps H) U, the
    matrix exponential of each link's momentum (scipy.linalg.expm)."""
    from scipy.linalg import expm
    U = np.asarray(U, dtype=np.complex128)
    H = np.asarray(H, dtype=np.complex128)
    out = np.empty_like(U)
    for mu in range(U.shape[0]):
        for x in range(U.shape[1]):
            out[mu, x] = expm(1j * float(eps) * H[mu, x]) @ U[mu, x]
    return out


def kinetic_energy(H) -> float:
    """H^2 / 2 of Eq. (1): half the sum over links of Tr H^2 (H Hermitian)."""
    H = np.asarray(H, dtype=np.complex128)
    return 0.5 * float(np.real(np.einsum("...ab,...ba->...", H, H).sum()))


def rational_apply(L, U, mass, alpha0, alpha, sigma, b, tol=1e-12, antiperiodic=True):
    """r(A) b_j = alpha0 b_j + sum_i alpha_i (A + sigma_i)^-1 b_j for every row of
    b (natural even-site [n][V][3]): a rational function of the even/odd
    operator in partial fractions, whose poles are the shifts of Eq. (2)
    (Sec. 2).  The oracle's multi-shift CG (with per-shift verification) to
    tol, then the sum, term by term in FP64."""
    V = _V(L)
    b = np.ascontiguousarray(b, dtype=np.complex128).reshape(-1, V, 3)
    out = np.empty_like(b)
    for j in range(b.shape[0]):
        X, st, _, _ = cg_multishift(L, U, mass, sigma, b[j], tol=tol, antiperiodic=antiperiodic)
        if st != 0:
            raise RuntimeError(f"oracle multi-shift CG failed with status {st}")
        y = float(alpha0) * b[j]
        for a, x in zip(alpha, X):
            y = y + float(a) * x
        out[j] = y
    return out


def action(L, alpha0, alpha, phi, X) -> float:
    """S = sum_j [alpha0 ||phi_j||^2 + sum_i alpha_i Re <phi_j, X_ij>]."""
    V = _V(L)
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.complex128).reshape(-1, V, 3)
    npf = phi.shape[0]
    X = _c128(np.asarray(X).reshape(npf, al.size, V, 3), (npf, al.size, V, 3))
    return float(_load().orc_action(_geom(L), npf, al.size, float(alpha0), _ptr(al),
                                    _ptr(phi), _ptr(X)))


def force(L, U, alpha, X, mode: int = 0, antiperiodic: bool = True) -> np.ndarray:
    """mode 0: TA(U M) per link; mode 1: M^dag (raw gradient).  Natural [4][V][3][3]."""
    V = _V(L)
    U = _c128(U, (4, V, 3, 3))
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.complex128)
    X = X.reshape(-1, al.size, V, 3)
    F = np.zeros((4, V, 3, 3), np.complex128)
    _load().orc_force(_geom(L), int(antiperiodic), _ptr(U), X.shape[0], al.size, _ptr(al),
                      _ptr(X), int(mode), _ptr(F))
    return F
