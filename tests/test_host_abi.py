"""CPU tests of the C ABI library and its host-side setup logic (no GPU
compute): symbol exports, LDU, option defaults, argument validation, the
stencil extraction, the Galerkin coarsening against a dense triple product,
the boundary-class compression and the coarse inverse."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle.ldu import coefficient_matrix, ldu
from oracle.tableau import tableau
from paper_2010_11377_amd import binding as B
from paper_2010_11377_amd import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_LIB = os.environ.get("IRK_HOST_TEST_LIB") or os.path.join(ROOT, "paper_2010_11377_amd",
                                                            "libirk_host_test.so")

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH),
                                reason="libirk.so not built (run __graft_entry__.build())")


def header_functions():
    with open(os.path.join(ROOT, "include", "irk.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irk_[a-z_]+)\s*\(", text)))


def test_all_header_symbols_exported():
    names = header_functions()
    assert "irk_setup" in names and "irk_step" in names and "irk_adjoint_step" in names
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B._PROTOS)


def test_default_options():
    o = B.default_options()
    assert (o.precision, o.precond, o.restart, o.max_iter, o.nu_pre, o.nu_post, o.coarse_max,
            o.vcycles, o.true_resid, o.reorth) == (0, 0, 40, 200, 2, 2, 64, 1, 1, 0)
    assert o.rtol == 1e-8
    assert o.side == B.IRK_RIGHT
    assert o.interp == B.IRK_INTERP_LINEAR
    assert o.graphs == 0
    assert o.coarse_ratio == 8.0
    assert o.smoother == B.SMOOTHER["rbgs"] and o.jacobi_omega == 0.8
    assert o.fuse_levels == 1


def test_status_strings():
    for code, name in [(0, "IRK_OK"), (-1, "IRK_E_INVALID"), (-2, "IRK_E_SINGULAR_PIVOT"),
                       (-3, "IRK_E_NOT_CONVERGED"), (-7, "IRK_E_OOM")]:
        assert B.status_string(code) == name


@pytest.mark.parametrize("family,s", [("gauss", 2), ("radau_iia", 3), ("radau_iia", 5),
                                      ("gauss", 7), ("lobatto_iiic", 4), ("radau_iia", 1)])
def test_irk_ldu_matches_oracle(family, s):
    A, b, c = tableau(family, s)
    A = np.ascontiguousarray(A)
    L = np.zeros((s, s))
    d = np.zeros(s)
    U = np.zeros((s, s))
    st = B.lib().irk_ldu(s, B.dptr(A), B.dptr(L), B.dptr(d), B.dptr(U))
    assert st == B.IRK_OK
    Lo, do, Uo = ldu(A)
    assert np.allclose(L, Lo, atol=1e-15) and np.allclose(d, do, atol=1e-15)
    assert np.allclose(U, Uo, atol=1e-14)


def test_irk_ldu_errors():
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    assert B.lib().irk_ldu(2, B.dptr(A), None, None, None) == B.IRK_E_SINGULAR_PIVOT
    assert B.lib().irk_ldu(9, B.dptr(np.eye(9)), None, None, None) == B.IRK_E_INVALID
    assert B.lib().irk_ldu(0, B.dptr(np.eye(1)), None, None, None) == B.IRK_E_INVALID


def _setup_status(A, b, K, h, grid, M=None, opt=None):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    tab = B.Butcher(A.shape[0], B.dptr(A), B.dptr(b), B.dptr(b))
    from paper_2010_11377_amd.solver import _csr_struct
    csr, keep = _csr_struct(*K)
    g = B.Grid(*grid)
    h_out = ctypes.c_void_p()
    o = opt if opt is not None else B.default_options()
    st = B.lib().irk_setup(ctypes.byref(h_out), ctypes.byref(tab),
                           ctypes.byref(M) if M is not None else None, ctypes.byref(csr), h,
                           ctypes.byref(g), ctypes.byref(o), None)
    return st, B.lib().irk_last_error(None).decode(), h_out


def test_setup_validation_before_any_device_work():
    """Argument errors are reported before the library touches the GPU."""
    n = 8
    K = problems.heat(n)
    A, b, c = tableau("radau_iia", 2)
    st, msg, h = _setup_status(A, b, K, -1.0, (n, n))
    assert st == B.IRK_E_INVALID and "h_t" in msg and not h.value
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n + 1))
    assert st == B.IRK_E_INVALID
    sing = np.array([[0.0, 0.5], [0.5, 0.5]])
    st, msg, _ = _setup_status(sing, b, K, 0.01, (n, n))
    assert st == B.IRK_E_SINGULAR_PIVOT
    opt = B.default_options()
    opt.restart = 0
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), opt=opt)
    assert st == B.IRK_E_INVALID and "restart" in msg
    opt = B.default_options()
    opt.side = 2
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), opt=opt)
    assert st == B.IRK_E_INVALID and "side" in msg
    opt = B.default_options()
    opt.graphs = 2
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), opt=opt)
    assert st == B.IRK_E_INVALID and "graphs" in msg
    opt = B.default_options()
    opt.smoother = 2
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), opt=opt)
    assert st == B.IRK_E_INVALID and "smoother" in msg
    opt = B.default_options()
    opt.smoother, opt.jacobi_omega = B.SMOOTHER["jacobi"], 1.5
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), opt=opt)
    assert st == B.IRK_E_INVALID and "jacobi_omega" in msg
    opt = B.default_options()
    opt.fuse_levels = 2
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), opt=opt)
    assert st == B.IRK_E_INVALID and "fuse_levels" in msg
    opt = B.default_options()
    opt.side, opt.precision = B.IRK_LEFT, B.IRK_MIXED
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), opt=opt)
    assert st == B.IRK_E_INVALID and "left" in msg
    # a coupling outside the 3x3 neighbourhood
    ip, ix, d = K
    ix = ix.copy()
    ip = ip.copy()
    ix[1] = 7 + 3 * n if ix[1] != 7 + 3 * n else ix[1]
    bad = (ip, np.sort(ix[:ip[1]]).tolist() + ix[ip[1]:].tolist(), d)
    bad = (ip, np.array(bad[1], dtype=np.int32), d)
    st, msg, _ = _setup_status(A, b, bad, 0.01, (n, n))
    assert st == B.IRK_E_INVALID and "stencil" in msg
    # unsorted columns in a row
    ix2 = K[1].copy()
    ix2[ip[5]], ix2[ip[5] + 1] = ix2[ip[5] + 1], ix2[ip[5]]
    st, msg, _ = _setup_status(A, b, (K[0], ix2, K[2]), 0.01, (n, n))
    assert st == B.IRK_E_INVALID and "sorted" in msg
    # non-finite entry
    d2 = K[2].copy()
    d2[3] = np.nan
    st, msg, _ = _setup_status(A, b, (K[0], K[1], d2), 0.01, (n, n))
    assert st == B.IRK_E_INVALID and "finite" in msg
    # mass matrices: wrong size, a coupling outside the 3 x 3 neighbourhood,
    # a zero diagonal entry
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), M=B.CSR())
    assert st == B.IRK_E_INVALID and "M and K differ" in msg
    from paper_2010_11377_amd.solver import _csr_struct
    mp, mi, md = problems.p1_heat(n)[0]
    far = mi.copy()
    far[mp[10] + 1] = (far[mp[10] + 1] + 3 * n) % (n * n)
    far_sorted = far.copy()
    for r in range(n * n):
        far_sorted[mp[r]:mp[r + 1]] = np.sort(far[mp[r]:mp[r + 1]])
    mcsr, keep = _csr_struct(mp, far_sorted, md)
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), M=mcsr)
    assert st == B.IRK_E_INVALID and msg.startswith("M:")
    zd = md.copy()
    zd[mp[10] + 3] = 0.0                 # row 10 (i = 2, j = 1): SW, S, W, C
    mcsr2, keep2 = _csr_struct(mp, mi, zd)
    st, msg, _ = _setup_status(A, b, K, 0.01, (n, n), M=mcsr2)
    assert st == B.IRK_E_INVALID and "diagonal" in msg


# ---------------------------------------------------------------- host library
@pytest.fixture(scope="module")
def H():
    if not os.path.exists(HOST_LIB):
        pytest.skip("host test library not built")
    L = ctypes.CDLL(HOST_LIB)
    pd = ctypes.POINTER(ctypes.c_double)
    pi = ctypes.POINTER(ctypes.c_int)
    L.irkh_csr_to_stencil.argtypes = [ctypes.c_int, pi, pi, pd, ctypes.c_int, ctypes.c_int, pd]
    L.irkh_galerkin.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, pd, pd]
    L.irkh_galerkin_constant.argtypes = [ctypes.c_int, ctypes.c_int, pd, pd]
    L.irkh_classify.argtypes = [ctypes.c_int, ctypes.c_int, pd, ctypes.c_double, pd]
    L.irkh_is_symmetric.argtypes = [ctypes.c_int, ctypes.c_int, pd, ctypes.c_double]
    L.irkh_dense_inverse.argtypes = [ctypes.c_int, ctypes.c_int, pd, pd]
    L.irkh_coefficient_matrix.argtypes = [ctypes.c_int, pd, ctypes.c_int, pd]
    return L


def stencil_of(H, K, n):
    ip, ix, d = [np.ascontiguousarray(a) for a in K]
    out = np.zeros(9 * n * n)
    rc = H.irkh_csr_to_stencil(n * n, ip.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                               ix.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), B.dptr(d), n, n,
                               B.dptr(out))
    assert rc == 0
    return out


def stencil_to_dense(st, nx, ny):
    N = nx * ny
    M = np.zeros((N, N))
    c = st.reshape(9, N)
    for j in range(ny):
        for i in range(nx):
            for k in range(9):
                dx, dy = k % 3 - 1, k // 3 - 1
                if 0 <= i + dx < nx and 0 <= j + dy < ny:
                    M[j * nx + i, (j + dy) * nx + i + dx] += c[k, j * nx + i]
                else:
                    assert c[k, j * nx + i] == 0.0
    return M


def transfers_dense(n, level):
    """The oracle's interpolation and 2x2 aggregation on hierarchy level
    ``level``, as dense matrices."""
    from oracle.amg import prolongation, restriction
    return prolongation(n, n, level).toarray(), restriction(n, n).toarray()


def test_stencil_roundtrip(H):
    n = 9
    K = problems.double_glazing(n, 0.01)[:3]
    st = stencil_of(H, K, n)
    assert np.allclose(stencil_to_dense(st, n, n), problems.to_dense(*K, n * n))


@pytest.mark.parametrize("which", ["heat", "dg", "kappa"])
def test_galerkin_is_dense_triple_product(H, which):
    n = 12
    if which == "heat":
        K = problems.heat(n)
    elif which == "dg":
        K = problems.double_glazing(n, 0.005)[:3]
    else:
        kn = np.exp(0.5 * np.random.default_rng(1).standard_normal((n + 2, n + 2)))
        K = problems.kappa_diffusion(kn)
    st = stencil_of(H, K, n)
    out = np.zeros(9 * (n // 2) ** 2)
    assert H.irkh_galerkin(n, n, 0, B.dptr(st), B.dptr(out)) == 0
    P, R = transfers_dense(n, 0)
    ref = R @ problems.to_dense(*K, n * n) @ P
    assert np.allclose(stencil_to_dense(out, n // 2, n // 2), ref, rtol=1e-13, atol=1e-12 * np.abs(ref).max())
    # two levels down: the product of products, with the level-1 weights
    out2 = np.zeros(9 * (n // 4) ** 2)
    assert H.irkh_galerkin(n // 2, n // 2, 1, B.dptr(out), B.dptr(out2)) == 0
    P2, R2 = transfers_dense(n // 2, 1)
    assert np.allclose(stencil_to_dense(out2, n // 4, n // 4), R2 @ ref @ P2, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("which", ["heat", "dg"])
def test_galerkin_constant_is_dense_triple_product(H, which):
    from oracle.amg import prolongation, restriction
    n = 12
    K = problems.heat(n) if which == "heat" else problems.double_glazing(n, 0.005)[:3]
    st = stencil_of(H, K, n)
    out = np.zeros(9 * (n // 2) ** 2)
    assert H.irkh_galerkin_constant(n, n, B.dptr(st), B.dptr(out)) == 0
    P = prolongation(n, n, 0, "constant").toarray()
    R = restriction(n, n).toarray()
    ref = R @ problems.to_dense(*K, n * n) @ P
    assert np.allclose(stencil_to_dense(out, n // 2, n // 2), ref, rtol=1e-13,
                       atol=1e-12 * np.abs(ref).max())


def test_classes(H):
    n = 32
    st = stencil_of(H, problems.heat(n), n)
    cls = np.zeros(81)
    assert H.irkh_classify(n, n, B.dptr(st), 1e-12, B.dptr(cls)) == 1
    assert H.irkh_is_symmetric(n, n, B.dptr(st), 1e-13) == 1
    cur, m, lev = st, n, 0
    while m >= 4:
        nxt = np.zeros(9 * (m // 2) ** 2)
        H.irkh_galerkin(m, m, lev, B.dptr(cur), B.dptr(nxt))
        cur, m, lev = nxt, m // 2, lev + 1
        assert H.irkh_classify(m, m, B.dptr(cur), 1e-12, B.dptr(cls)) == 1
    dg = stencil_of(H, problems.double_glazing(n, 0.005)[:3], n)
    assert H.irkh_classify(n, n, B.dptr(dg), 1e-12, B.dptr(cls)) == 0
    assert H.irkh_is_symmetric(n, n, B.dptr(dg), 1e-13) == 0


def test_dense_inverse(H):
    n = 6
    st = stencil_of(H, problems.double_glazing(n, 0.05)[:3], n)
    inv = np.zeros((n * n) ** 2)
    assert H.irkh_dense_inverse(n, n, B.dptr(st), B.dptr(inv)) == 0
    ref = np.linalg.inv(stencil_to_dense(st, n, n))
    assert np.allclose(inv.reshape(n * n, n * n), ref, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kind,name", [(0, "LD"), (1, "DU"), (2, "GSL"), (3, "J")])
def test_coefficient_matrices(H, kind, name):
    for family, s in [("radau_iia", 3), ("gauss", 7), ("lobatto_iiic", 4)]:
        A, b, c = tableau(family, s)
        A = np.ascontiguousarray(A)
        out = np.zeros(s * s)
        assert H.irkh_coefficient_matrix(s, B.dptr(A), kind, B.dptr(out)) == 0
        assert np.allclose(out.reshape(s, s), coefficient_matrix(A, name), atol=1e-15)
