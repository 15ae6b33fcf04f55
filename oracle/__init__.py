"""Plain FP64 CPU oracle for Galerkin BEM entries (arXiv 1510.07244).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  It
shares no code with the HIP path; the only module both sides use is
``bem_inputs`` (seeded meshes and index samples, no method arithmetic).

The numerical work lives in ``oracle.c`` (see its header for the formulas
and the paper passages they follow); this module marshals numpy arrays.
"""
import ctypes
import os

import numpy as np

from .build import LIB, NATIVE_LIB, build

_lib = None
_lib_path = LIB

LAPLACE, HELMHOLTZ = 0, 1
SLP, DLP = 0, 1
RULE_DUFFY, RULE_TRI7 = 0, 1
DISJOINT, VERTEX, EDGE, IDENTICAL = 0, 1, 2, 3


def use_native_build():
    """Switch to an ``-O3 -march=native`` build of the oracle compiled on this
    host (same source; used to time the CPU baseline)."""
    global _lib, _lib_path
    build(native=True)
    _lib, _lib_path = None, NATIVE_LIB


def use_library(path):
    """Load the oracle from another build of the same source (the tests run
    an address- and undefined-behaviour-sanitized build through this)."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_lib_path):
            build()
        L = ctypes.CDLL(_lib_path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oracle_gauss01.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_tri7.argtypes = [dp, dp]
        L.oracle_shared_vertices.argtypes = [ip, ctypes.c_int, ctypes.c_int]
        L.oracle_ss_nregions.argtypes = [ctypes.c_int]
        L.oracle_ss_rule.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.oracle_ss_rule.restype = ctypes.c_long
        L.oracle_entries.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_long, ip, ip, dp]
        L.oracle_green_matrix.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ip,
                                          ctypes.c_int, dp, dp, dp, ctypes.c_double, dp]
        L.oracle_inverse.argtypes = [ctypes.c_int, dp, dp]
        L.oracle_contract.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, dp, dp]
        L.oracle_interp_basis.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ip, ip,
                                          dp, dp]
        L.oracle_p1_pairs.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_long, ip, ip, dp]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def gauss01(q):
    """q-point Gauss-Legendre rule on [0,1] (nodes increasing)."""
    x = np.zeros(q)
    w = np.zeros(q)
    if lib().oracle_gauss01(q, _d(x), _d(w)):
        raise ValueError("bad order")
    return x, w


def tri7():
    """Seven-point degree-5 triangle rule: barycentric (7,3), weights (7,)."""
    b = np.zeros((7, 3))
    w = np.zeros(7)
    lib().oracle_tri7(_d(b), _d(w))
    return b, w


def shared_vertices(tri, i, j):
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    return lib().oracle_shared_vertices(_i(tri), int(i), int(j))


def ss_rule(case, q):
    """Sauter-Schwab rule of the case (3 identical, 2 edge, 1 vertex) in
    reference coordinates: pts (P,4) = (x^1, x^2, y^1, y^2), weights (P,)."""
    nreg = lib().oracle_ss_nregions(case)
    n = nreg * q ** 4
    pts = np.zeros((n, 4))
    w = np.zeros(n)
    got = lib().oracle_ss_rule(case, q, _d(pts), _d(w))
    if got != n:
        raise ValueError("bad rule")
    return pts, w


def entries(v, tri, rows, cols, kernel=LAPLACE, layer=SLP, kappa=0.0,
            rule=RULE_DUFFY, q_reg=4, q_sing=4):
    """Galerkin entries G(rows[k], cols[k]) as complex128 (Laplace: Im = 0)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int32).ravel()
    cols = np.ascontiguousarray(cols, dtype=np.int32).ravel()
    if rows.shape != cols.shape:
        raise ValueError("rows/cols shape mismatch")
    out = np.zeros(2 * rows.size)
    rc = lib().oracle_entries(_d(v), v.shape[0], _i(tri), tri.shape[0], kernel, layer,
                              float(kappa), rule, q_reg, q_sing, rows.size, _i(rows),
                              _i(cols), _d(out))
    if rc:
        raise ValueError("oracle_entries: invalid arguments")
    return out[0::2] + 1j * out[1::2]


def block(v, tri, rows, cols, **op):
    """Dense block G[rows x cols] (row-major numpy array)."""
    rows = np.asarray(rows, dtype=np.int32)
    cols = np.asarray(cols, dtype=np.int32)
    R, C = np.meshgrid(rows, cols, indexing="ij")
    return entries(v, tri, R.ravel(), C.ravel(), **op).reshape(rows.size, cols.size)


def p1_pairs(v, tri, rows, cols, kernel=LAPLACE, layer=SLP, kappa=0.0, q_reg=4, q_sing=4):
    """3 x 3 local matrices of piecewise-linear bases, (n, 3, 3) complex128:
    L[k, a, b] = int int lambda_a(x) kernel(x, y) mu_b(y) over triangles
    rows[k] and cols[k] (a, b: their vertices in mesh order)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int32).ravel()
    cols = np.ascontiguousarray(cols, dtype=np.int32).ravel()
    if rows.shape != cols.shape:
        raise ValueError("rows/cols shape mismatch")
    out = np.zeros(18 * rows.size)
    if lib().oracle_p1_pairs(_d(v), v.shape[0], _i(tri), tri.shape[0], kernel, layer,
                             float(kappa), q_reg, q_sing, rows.size, _i(rows), _i(cols), _d(out)):
        raise ValueError("oracle_p1_pairs: invalid arguments")
    return (out[0::2] + 1j * out[1::2]).reshape(rows.size, 3, 3)


def p1_block(v, tri, row_vertices, col_vertices, **op):
    """Dense block of the piecewise-linear Galerkin matrix: entry (v, w) is
    the sum of L[a, b] over the triangles a around vertex v and b around
    vertex w, at the positions of v in a and of w in b (complex128)."""
    tri = np.asarray(tri)
    star = {}
    for t, t3 in enumerate(tri):
        for k in range(3):
            star.setdefault(int(t3[k]), []).append((t, k))
    rv = [int(x) for x in row_vertices]
    cv = [int(x) for x in col_vertices]
    ta = sorted({t for x in rv for t, _ in star.get(x, [])})
    tb = sorted({t for x in cv for t, _ in star.get(x, [])})
    pos_a = {t: i for i, t in enumerate(ta)}
    pos_b = {t: i for i, t in enumerate(tb)}
    R, C = np.meshgrid(np.array(ta, dtype=np.int32), np.array(tb, dtype=np.int32), indexing="ij")
    L = p1_pairs(v, tri, R.ravel(), C.ravel(), **op).reshape(len(ta), len(tb), 3, 3)
    G = np.zeros((len(rv), len(cv)), dtype=np.complex128)
    for i, x in enumerate(rv):
        for j, y in enumerate(cv):
            s = 0.0
            for a, k in star.get(x, []):
                for b, l in star.get(y, []):
                    s += L[pos_a[a], pos_b[b], k, l]
            G[i, j] = s
    return G


def green_matrix(v, tri, rows, z, zn, zw, delta, kernel=LAPLACE, kappa=0.0, side=0, q=4):
    """Green quadrature matrix (len(rows), 2m) complex128 of one cluster."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    z = np.ascontiguousarray(z, dtype=np.float64)
    zn = np.ascontiguousarray(zn, dtype=np.float64)
    zw = np.ascontiguousarray(zw, dtype=np.float64)
    m = zw.size
    out = np.zeros(2 * rows.size * 2 * m)
    rc = lib().oracle_green_matrix(_d(v), v.shape[0], _i(tri), tri.shape[0], kernel,
                                   float(kappa), side, q, rows.size, _i(rows), m, _d(z),
                                   _d(zn), _d(zw), float(delta), _d(out))
    if rc:
        raise ValueError("oracle_green_matrix: invalid arguments")
    c = out[0::2] + 1j * out[1::2]
    return c.reshape(2 * m, rows.size).T


def _cplx_colmajor(A):
    """complex128 matrix -> interleaved column-major float64 buffer."""
    A = np.asarray(A, dtype=np.complex128)
    return np.ascontiguousarray(A.T.ravel()).view(np.float64)


def _from_colmajor(buf, n, k):
    return buf.view(np.complex128).reshape(k, n).T


def inverse(M):
    """Inverse of a square matrix by Gauss-Jordan elimination (complex128)."""
    M = np.asarray(M)
    k = M.shape[0]
    P = np.zeros(2 * k * k)
    if lib().oracle_inverse(k, _d(_cplx_colmajor(M)), _d(P)):
        raise ValueError("singular pivot block")
    return _from_colmajor(P, k, k)


def contract(A, tau, P):
    """V = A[:, tau] P by one sum per entry (complex128)."""
    A = np.asarray(A)
    n, acols = A.shape
    tau = np.ascontiguousarray(tau, dtype=np.int32)
    k = tau.size
    V = np.zeros(2 * n * k)
    if lib().oracle_contract(n, acols, _d(_cplx_colmajor(A)), k, _i(tau),
                             _d(_cplx_colmajor(P)), _d(V)):
        raise ValueError("oracle_contract: invalid arguments")
    return _from_colmajor(V, n, k)


def interp_basis(A, prow, tau):
    """Interpolation basis V = A[:, tau] A[prow, tau]^{-1} and the inverse
    (complex128)."""
    A = np.asarray(A)
    n, acols = A.shape
    prow = np.ascontiguousarray(prow, dtype=np.int32)
    tau = np.ascontiguousarray(tau, dtype=np.int32)
    k = tau.size
    V = np.zeros(2 * n * k)
    P = np.zeros(2 * k * k)
    if lib().oracle_interp_basis(n, acols, _d(_cplx_colmajor(A)), k, _i(prow), _i(tau), _d(V),
                                 _d(P)):
        raise ValueError("oracle_interp_basis: invalid arguments or singular pivot block")
    return _from_colmajor(V, n, k), _from_colmajor(P, k, k)


def num_threads():
    """OpenMP threads the oracle's loops use."""
    return int(lib().oracle_num_threads())


def set_threads(n):
    """Threads of the oracle's following parallel loops."""
    lib().oracle_set_threads(int(n))
