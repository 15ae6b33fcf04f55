"""Thin Python binding of the MI355X Galerkin BEM assembly library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libbem.so`` (C-ABI declared in ``include/bem.h``).  PyTorch
provides device memory and streams.  There is no CPU fallback: importing the
binding fails loudly when the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem.so")

BEM_OK, BEM_EINVAL, BEM_ENOMEM, BEM_EDEVICE, BEM_EUNSUPPORTED, BEM_ENONFINITE = 0, -1, -2, -3, -4, -5
LAPLACE, HELMHOLTZ = 0, 1
SLP, DLP = 0, 1
# bem_batch.layers
BATCH_OP_LAYER, BATCH_SLP, BATCH_DLP, BATCH_BOTH = 0, 1, 2, 3
PLAIN_FP64, MIXED = 0, 1
RULE_DUFFY, RULE_TRI7 = 0, 1
MAX_ORDER = 12
NOALLOC_MAX_TRI = 32768  # largest mesh of bem_assemble_nearfield_noalloc

_ERRNAMES = {BEM_EINVAL: "EINVAL", BEM_ENOMEM: "ENOMEM", BEM_EDEVICE: "EDEVICE",
             BEM_EUNSUPPORTED: "EUNSUPPORTED", BEM_ENONFINITE: "ENONFINITE"}


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class bem_mesh(ctypes.Structure):
    _fields_ = [("v", ctypes.c_void_p), ("nv", ctypes.c_int32),
                ("tri", ctypes.c_void_p), ("nt", ctypes.c_int32)]


class bem_op(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("layer", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("regular_rule", ctypes.c_int32),
                ("q_regular", ctypes.c_int32), ("q_singular", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("near_singular_ratio", ctypes.c_double),
                ("reserved", ctypes.c_int32 * 4)]


class bem_blocks(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("row_ptr", ctypes.c_void_p), ("row_idx", ctypes.c_void_p),
                ("row_len", ctypes.c_int64), ("col_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("col_len", ctypes.c_int64),
                ("out_off", ctypes.c_void_p), ("mirror_off", ctypes.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1510_07244_amd/build.py "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.bem_create.argtypes = [ctypes.POINTER(P), ctypes.c_int]
    L.bem_destroy.argtypes = [P]
    L.bem_destroy.restype = None
    L.bem_last_error.argtypes = [P]
    L.bem_last_error.restype = ctypes.c_char_p
    L.bem_check.argtypes = [P, P]
    for name in ("bem_assemble_nearfield", "bem_assemble_coupling",
                 "bem_assemble_nearfield_noalloc"):
        getattr(L, name).argtypes = [P, ctypes.POINTER(bem_mesh), ctypes.POINTER(bem_op),
                                     ctypes.POINTER(bem_blocks), P, ctypes.c_int64, P]
    L.bem_assemble_nearfield_both.argtypes = [P, ctypes.POINTER(bem_mesh), ctypes.POINTER(bem_op),
                                              ctypes.POINTER(bem_blocks), P, P, ctypes.c_int64, P]
    L.bem_eval_entries.argtypes = [P, ctypes.POINTER(bem_mesh), ctypes.POINTER(bem_op),
                                   ctypes.c_int64, P, P, P, P]
    L.bem_cluster_tree.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, P, P, P, P, P, P, P]
    L.bem_block_tree.argtypes = [ctypes.c_int32, P, P, ctypes.c_double, ctypes.c_int32,
                                 P, P, P, P]
    return L


_lib = _load()


def lib():
    return _lib


def make_op(kernel=LAPLACE, layer=SLP, precision=PLAIN_FP64, regular_rule=RULE_DUFFY,
            q_regular=4, q_singular=4, kappa=0.0, near_singular_ratio=0.0):
    return bem_op(kernel, layer, precision, regular_rule, q_regular, q_singular, float(kappa),
                  float(near_singular_ratio), (ctypes.c_int32 * 4)(0, 0, 0, 0))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(0)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


class Mesh:
    """Device mesh: v (nv,3) float64 and tri (nt,3) int32 CUDA tensors."""

    def __init__(self, v, tri):
        import torch
        self.v = v.to(device="cuda", dtype=torch.float64).contiguous()
        self.tri = tri.to(device="cuda", dtype=torch.int32).contiguous()
        self.c = bem_mesh(_ptr(self.v), self.v.shape[0], _ptr(self.tri), self.tri.shape[0])


class Blocks:
    """Device block list (CSR row/column triangle lists and output offsets)."""

    def __init__(self, row_ptr, row_idx, col_ptr, col_idx, out_off, mirror_off=None):
        import torch
        dev = dict(device="cuda")
        self.row_ptr = torch.as_tensor(row_ptr, dtype=torch.int32).to(**dev).contiguous()
        self.row_idx = torch.as_tensor(row_idx, dtype=torch.int32).to(**dev).contiguous()
        self.col_ptr = torch.as_tensor(col_ptr, dtype=torch.int32).to(**dev).contiguous()
        self.col_idx = torch.as_tensor(col_idx, dtype=torch.int32).to(**dev).contiguous()
        self.out_off = torch.as_tensor(out_off, dtype=torch.int64).to(**dev).contiguous()
        self.mirror_off = (None if mirror_off is None else
                           torch.as_tensor(mirror_off, dtype=torch.int64).to(**dev).contiguous())
        self.n = self.out_off.numel()
        self.c = bem_blocks(self.n, _ptr(self.row_ptr), _ptr(self.row_idx), self.row_idx.numel(),
                            _ptr(self.col_ptr), _ptr(self.col_idx), self.col_idx.numel(),
                            _ptr(self.out_off),
                            None if self.mirror_off is None else _ptr(self.mirror_off))

    @classmethod
    def from_lists(cls, rows, cols):
        """Blocks from lists of row / column index arrays; outputs packed back
        to back.  Returns (blocks, total number of entries)."""
        import numpy as np
        rp = np.zeros(len(rows) + 1, dtype=np.int64)
        cp = np.zeros(len(cols) + 1, dtype=np.int64)
        rp[1:] = np.cumsum([len(r) for r in rows])
        cp[1:] = np.cumsum([len(c) for c in cols])
        sizes = np.array([len(r) * len(c) for r, c in zip(rows, cols)], dtype=np.int64)
        off = np.zeros(len(rows), dtype=np.int64)
        off[1:] = np.cumsum(sizes)[:-1]
        cat = lambda xs: np.concatenate([np.asarray(x, dtype=np.int32) for x in xs]) if xs else np.zeros(0, np.int32)
        b = cls(rp.astype(np.int32), cat(rows), cp.astype(np.int32), cat(cols), off)
        return b, int(sizes.sum())


class Context:
    """A library context on one device (``bem_create``)."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        rc = _lib.bem_create(ctypes.byref(h), int(device))
        if rc:
            raise BemError(rc, "bem_create failed")
        self.h = h

    def close(self):
        if self.h:
            _lib.bem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self):
        return _lib.bem_last_error(self.h).decode()

    def _rc(self, rc):
        if rc:
            raise BemError(rc, self.last_error())

    def check(self, stream=None):
        """bem_check: synchronise and raise on a device-side error flag."""
        self._rc(_lib.bem_check(self.h, _stream(stream)))

    def assemble_nearfield(self, mesh, op, blocks, out, stream=None):
        self._rc(_lib.bem_assemble_nearfield(self.h, ctypes.byref(mesh.c), ctypes.byref(op),
                                             ctypes.byref(blocks.c), _ptr(out), out.numel(),
                                             _stream(stream)))

    def assemble_nearfield_noalloc(self, mesh, op, blocks, out, stream=None):
        """bem_assemble_nearfield_noalloc: as assemble_nearfield, allocating
        nothing (geometry in the library's fixed per-GPU array; the orders'
        quadrature tables must exist on the context already)."""
        self._rc(_lib.bem_assemble_nearfield_noalloc(self.h, ctypes.byref(mesh.c),
                                                     ctypes.byref(op), ctypes.byref(blocks.c),
                                                     _ptr(out), out.numel(), _stream(stream)))

    def assemble_nearfield_both(self, mesh, op, blocks, out_slp, out_dlp, stream=None):
        """bem_assemble_nearfield_both: single layer to out_slp, double layer
        to out_dlp (same length and type), one pass."""
        if out_slp.numel() != out_dlp.numel() or out_slp.dtype != out_dlp.dtype:
            raise ValueError("out_slp and out_dlp must have the same length and dtype")
        self._rc(_lib.bem_assemble_nearfield_both(self.h, ctypes.byref(mesh.c), ctypes.byref(op),
                                                  ctypes.byref(blocks.c), _ptr(out_slp),
                                                  _ptr(out_dlp), out_slp.numel(), _stream(stream)))

    def assemble_coupling(self, mesh, op, pivots, out, stream=None):
        self._rc(_lib.bem_assemble_coupling(self.h, ctypes.byref(mesh.c), ctypes.byref(op),
                                            ctypes.byref(pivots.c), _ptr(out), out.numel(),
                                            _stream(stream)))

    def eval_entries(self, mesh, op, rows, cols, out, stream=None):
        self._rc(_lib.bem_eval_entries(self.h, ctypes.byref(mesh.c), ctypes.byref(op),
                                       rows.numel(), _ptr(rows), _ptr(cols), _ptr(out),
                                       _stream(stream)))


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class ClusterTree:
    """Host cluster tree (``bem_cluster_tree``): perm, begin/end, sons, level,
    box (lo, hi); ``idx(c)`` gives the triangle ids of cluster c."""

    def __init__(self, v, tri, leaf=64):
        import numpy as np
        v = np.ascontiguousarray(v, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        nt = tri.shape[0]
        cap = max(2 * nt - 1, 1)
        self.perm = np.zeros(nt, dtype=np.int32)
        ncl = ctypes.c_int32()
        self.begin = np.zeros(cap, dtype=np.int32)
        self.end = np.zeros(cap, dtype=np.int32)
        self.sons = np.zeros(2 * cap, dtype=np.int32)
        self.level = np.zeros(cap, dtype=np.int32)
        self.box = np.zeros(6 * cap, dtype=np.float64)
        rc = _lib.bem_cluster_tree(_np_ptr(v), v.shape[0], _np_ptr(tri), nt, int(leaf), cap,
                                   _np_ptr(self.perm), ctypes.byref(ncl), _np_ptr(self.begin),
                                   _np_ptr(self.end), _np_ptr(self.sons), _np_ptr(self.level),
                                   _np_ptr(self.box))
        if rc:
            raise BemError(rc, "bem_cluster_tree failed")
        n = ncl.value
        self.n = n
        self.begin, self.end, self.level = self.begin[:n], self.end[:n], self.level[:n]
        self.sons = self.sons[:2 * n].reshape(n, 2)
        self.box = self.box[:6 * n].reshape(n, 6)

    def idx(self, c):
        return self.perm[self.begin[c]:self.end[c]]

    def is_leaf(self, c):
        return self.sons[c, 0] < 0


def block_tree(ct, eta=2.0):
    """(near, far) lists of (t, s) cluster pairs (``bem_block_tree``)."""
    import numpy as np
    cap = 1024
    while True:
        near = np.zeros(2 * cap, dtype=np.int32)
        far = np.zeros(2 * cap, dtype=np.int32)
        nn, nf = ctypes.c_int32(), ctypes.c_int32()
        sons = np.ascontiguousarray(ct.sons.ravel())
        box = np.ascontiguousarray(ct.box.ravel())
        rc = _lib.bem_block_tree(ct.n, _np_ptr(sons), _np_ptr(box), float(eta), cap,
                                 _np_ptr(near), ctypes.byref(nn), _np_ptr(far), ctypes.byref(nf))
        if rc == 0:
            return near[:2 * nn.value].reshape(-1, 2), far[:2 * nf.value].reshape(-1, 2)
        if max(nn.value, nf.value) <= cap:
            raise BemError(rc, "bem_block_tree failed")
        cap = max(nn.value, nf.value)


def out_dtype(op):
    """torch dtype of one output entry for an operator."""
    import torch
    if op.precision == MIXED:
        return torch.complex64 if op.kernel == HELMHOLTZ else torch.float32
    return torch.complex128 if op.kernel == HELMHOLTZ else torch.float64


def _setup_bases_api():
    P = ctypes.c_void_p
    _lib.bem_green_points.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, P, P, P]
    _lib.bem_aca.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, ctypes.c_int32, P,
                             ctypes.c_double, ctypes.c_int32, P, P, P, P]
    _lib.bem_green_matrix.argtypes = [P, ctypes.POINTER(bem_mesh), ctypes.POINTER(bem_op),
                                      ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int64,
                                      ctypes.c_int32, P, P, P, P, P, P, ctypes.c_int64,
                                      ctypes.c_int32, P]
    _lib.bem_basis_contract.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32,
                                        P, P, P, P, ctypes.c_int32, ctypes.c_int64, P, P,
                                        ctypes.c_int64, ctypes.c_int32, P]
    _lib.bem_pivot_inverse.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32,
                                       P, P, P, P, ctypes.c_int32, ctypes.c_int64, P, P]


_setup_bases_api()


def green_points(boxes, qg):
    """``bem_green_points``: boxes (ncl, 6) -> z (ncl, m, 3), zn, zw (ncl, m), delta."""
    import numpy as np
    boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 6)
    ncl = boxes.shape[0]
    m = 6 * qg * qg
    z = np.zeros((ncl, m, 3))
    zn = np.zeros((ncl, m, 3))
    zw = np.zeros((ncl, m))
    delta = np.zeros(ncl)
    rc = _lib.bem_green_points(ncl, _np_ptr(boxes), int(qg), _np_ptr(z), _np_ptr(zn),
                               _np_ptr(zw), _np_ptr(delta))
    if rc:
        raise BemError(rc, "bem_green_points failed")
    return z, zn, zw, delta


def aca(A, a_off, nrows, ncols, eps, max_rank, is_complex=False, inverse=True):
    """``bem_aca`` on packed host matrices (float64 array; complex as
    interleaved pairs).  Returns rank, piv_rows, piv_cols, pinv (None when
    inverse is False: pivots only)."""
    import numpy as np
    A = np.ascontiguousarray(A)
    a_off = np.ascontiguousarray(a_off, dtype=np.int64)
    nrows = np.ascontiguousarray(nrows, dtype=np.int32)
    nmat = nrows.size
    rank = np.zeros(nmat, dtype=np.int32)
    piv_rows = np.zeros((nmat, max_rank), dtype=np.int32)
    piv_cols = np.zeros((nmat, max_rank), dtype=np.int32)
    pinv = (np.zeros((nmat, max_rank * max_rank * (2 if is_complex else 1)), dtype=np.float64)
            if inverse else None)
    rc = _lib.bem_aca(nmat, _np_ptr(a_off), _np_ptr(nrows), int(ncols), int(bool(is_complex)),
                      _np_ptr(A), float(eps), int(max_rank), _np_ptr(rank), _np_ptr(piv_rows),
                      _np_ptr(piv_cols), _np_ptr(pinv) if inverse else ctypes.c_void_p(0))
    if rc:
        raise BemError(rc, "bem_aca failed")
    return rank, piv_rows, piv_cols, pinv


def _context_green_matrix(self, mesh, op, side, row_ptr, row_idx, z, zn, zw, delta, out_off,
                          out, max_rows=64, stream=None):
    m = zw.shape[-1] if zw.dim() > 1 else zw.numel()
    self._rc(_lib.bem_green_matrix(self.h, ctypes.byref(mesh.c), ctypes.byref(op), int(side),
                                   out_off.numel(), _ptr(row_ptr), _ptr(row_idx), row_idx.numel(),
                                   int(m), _ptr(z), _ptr(zn), _ptr(zw), _ptr(delta),
                                   _ptr(out_off), _ptr(out), out.numel(), int(max_rows),
                                   _stream(stream)))


def _context_basis_contract(self, is_complex, nrows, rank, max_rank, piv_cols, pinv, A, a_off,
                            acols, V, v_off, max_rows=64, stream=None):
    self._rc(_lib.bem_basis_contract(self.h, int(bool(is_complex)), nrows.numel(), _ptr(nrows),
                                     _ptr(rank), int(max_rank), _ptr(piv_cols), _ptr(pinv),
                                     _ptr(A), _ptr(a_off), int(acols), A.numel(), _ptr(V),
                                     _ptr(v_off), V.numel(), int(max_rows), _stream(stream)))


def _context_valu_peak(self, fp64=True, stream=None):
    """bem_valu_peak: measured vector-ALU peak (TFLOP/s) of the context's GPU."""
    _lib.bem_valu_peak.argtypes = [ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]
    r = ctypes.c_double()
    self._rc(_lib.bem_valu_peak(self.h, int(bool(fp64)), ctypes.byref(r), _stream(stream)))
    return r.value


Context.valu_peak = _context_valu_peak


def _setup_h2mv_api():
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    _lib.bem_gemv_grouped.argtypes = [P, i32, i32, i32, P, P, P, i64, i32, P, P, i64, P, P, i64,
                                      P, i64, P, i64, P]
    _lib.bem_vec_dot.argtypes = [P, i32, i32, i64, P, P, P, P]
    _lib.bem_vec_axpby.argtypes = [P, i32, i64, f64, f64, P, f64, f64, P, P]
    _lib.bem_mass_apply.argtypes = [P, ctypes.POINTER(bem_mesh), i32, f64, f64, P, P, P]
    _lib.bem_cg_step.argtypes = [P, i64, P, P, P, P, P, P]


_setup_h2mv_api()


def _n(t):
    """Entries of a real or complex tensor."""
    return t.numel()


def _context_gemv_grouped(self, trans, grp_ptr, out_ptr, out_idx, in_ptr, in_idx, a_off, A, x, y,
                          stream=None):
    """bem_gemv_grouped on device tensors (complex when A is)."""
    cplx = A.is_complex()
    self._rc(_lib.bem_gemv_grouped(self.h, int(cplx), int(bool(trans)), grp_ptr.numel() - 1,
                                   _ptr(grp_ptr), _ptr(out_ptr), _ptr(out_idx), out_idx.numel(),
                                   in_ptr.numel() - 1, _ptr(in_ptr), _ptr(in_idx), in_idx.numel(),
                                   _ptr(a_off), _ptr(A), _n(A), _ptr(x), _n(x), _ptr(y), _n(y),
                                   _stream(stream)))


def _context_vec_dot(self, x, y, out, conj=True, stream=None):
    """bem_vec_dot into the device double[2] `out`."""
    self._rc(_lib.bem_vec_dot(self.h, int(x.is_complex()), int(bool(conj)), _n(x), _ptr(x), _ptr(y),
                              _ptr(out), _stream(stream)))


def _context_vec_axpby(self, alpha, x, beta, y, stream=None):
    """bem_vec_axpby: y = alpha x + beta y (alpha, beta Python numbers)."""
    a, b = complex(alpha), complex(beta)
    self._rc(_lib.bem_vec_axpby(self.h, int(x.is_complex()), _n(x), a.real, a.imag, _ptr(x),
                                b.real, b.imag, _ptr(y), _stream(stream)))


def _context_cg_step(self, state, x, r, p, q, stream=None):
    """bem_cg_step: one conjugate-gradient step with its scalars in the
    device double[10] `state` (layout in include/bem.h)."""
    self._rc(_lib.bem_cg_step(self.h, _n(x), _ptr(state), _ptr(x), _ptr(r), _ptr(p), _ptr(q),
                              _stream(stream)))


def _context_mass_apply(self, mesh, c, x, y, stream=None):
    """bem_mass_apply: y += c M x."""
    c = complex(c)
    self._rc(_lib.bem_mass_apply(self.h, ctypes.byref(mesh.c), int(x.is_complex()), c.real, c.imag,
                                 _ptr(x), _ptr(y), _stream(stream)))


def _setup_p1_api():
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    _lib.bem_p1_pairs.argtypes = [P, ctypes.POINTER(bem_mesh), ctypes.POINTER(bem_op), i64, P, P,
                                  P, P]
    _lib.bem_p1_gather.argtypes = [P, i32, i32, P, P, P, i64, i32, P, P, P, i64, i32, i32, P, P,
                                   P]


_setup_p1_api()


def _context_p1_pairs(self, mesh, op, rows, cols, out, stream=None):
    """bem_p1_pairs: out (9 n entries) = local 3 x 3 matrices of the pairs."""
    self._rc(_lib.bem_p1_pairs(self.h, ctypes.byref(mesh.c), ctypes.byref(op), rows.numel(),
                               _ptr(rows), _ptr(cols), _ptr(out), _stream(stream)))


def _context_p1_gather(self, rs_ptr, rs_tri, rs_loc, cs_ptr, cs_tri, cs_loc, ntr, ntc, local,
                       out, stream=None):
    """bem_p1_gather: dense vertex block from the pairs' local matrices."""
    self._rc(_lib.bem_p1_gather(self.h, int(local.is_complex()), rs_ptr.numel() - 1, _ptr(rs_ptr),
                                _ptr(rs_tri), _ptr(rs_loc), rs_tri.numel(), cs_ptr.numel() - 1,
                                _ptr(cs_ptr), _ptr(cs_tri), _ptr(cs_loc), cs_tri.numel(),
                                int(ntr), int(ntc), _ptr(local), _ptr(out), _stream(stream)))


Context.p1_pairs = _context_p1_pairs
Context.p1_gather = _context_p1_gather
Context.gemv_grouped = _context_gemv_grouped
Context.vec_dot = _context_vec_dot
Context.vec_axpby = _context_vec_axpby
Context.cg_step = _context_cg_step
Context.mass_apply = _context_mass_apply
def _context_pivot_inverse(self, is_complex, nrows, rank, max_rank, piv_rows, piv_cols, A, a_off,
                           acols, pinv, stream=None):
    self._rc(_lib.bem_pivot_inverse(self.h, int(bool(is_complex)), nrows.numel(), _ptr(nrows),
                                    _ptr(rank), int(max_rank), _ptr(piv_rows), _ptr(piv_cols),
                                    _ptr(A), _ptr(a_off), int(acols), A.numel(), _ptr(pinv),
                                    _stream(stream)))


Context.pivot_inverse = _context_pivot_inverse
Context.green_matrix = _context_green_matrix
Context.basis_contract = _context_basis_contract


# ------------------------------------------------------------ batched plans
class bem_batch(ctypes.Structure):
    _fields_ = [("mesh", ctypes.POINTER(bem_mesh)), ("blocks", ctypes.POINTER(bem_blocks)),
                ("coupling", ctypes.c_int32), ("layers", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("out_len", ctypes.c_int64),
                ("out2", ctypes.c_void_p)]


def _batch(entry):
    """bem_batch of a plan entry (mesh, blocks, out, coupling[, layers[, out2]])."""
    mesh, blocks, out, coupling = entry[:4]
    layers = int(entry[4]) if len(entry) > 4 else BATCH_OP_LAYER
    out2 = entry[5] if len(entry) > 5 else None
    return bem_batch(ctypes.pointer(mesh.c), ctypes.pointer(blocks.c), int(bool(coupling)), layers,
                     _ptr(out), out.numel(), _ptr(out2))


class bem_tune(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_cols", ctypes.c_int32), ("x_chunk", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("granularity", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2),
                ("tuned_ms", ctypes.c_double)]


def _setup_plan_api():
    P = ctypes.c_void_p
    _lib.bem_plan_batched.argtypes = [P, ctypes.POINTER(bem_op), ctypes.c_int32,
                                      ctypes.POINTER(bem_batch), ctypes.POINTER(bem_tune),
                                      ctypes.c_char_p, P, ctypes.POINTER(P)]
    _lib.bem_run_batched.argtypes = [P, P]
    _lib.bem_plan_tiles.argtypes = [P]
    _lib.bem_plan_tiles.restype = ctypes.c_int64
    _lib.bem_plan_destroy.argtypes = [P]
    _lib.bem_plan_destroy.restype = None
    _lib.bem_autotune.argtypes = [P, ctypes.POINTER(bem_op), ctypes.c_int32,
                                  ctypes.POINTER(bem_batch), ctypes.POINTER(bem_tune),
                                  ctypes.c_char_p, P]


_setup_plan_api()


def autotune(ctx, op, entries, tune=None, cache=None, stream=None):
    """``bem_autotune``: time the launch configurations of a batch (entries
    as for Plan), store the winner in the cache file, keep no plan.
    Returns the chosen configuration."""
    entries = list(entries)
    c = (bem_batch * max(len(entries), 1))()
    for k, e in enumerate(entries):
        c[k] = _batch(e)
    t = dict(tune or {})
    cfg = bem_tune(int(t.get("grid", 0)), int(t.get("tile_rows", 0)), int(t.get("tile_cols", 0)),
                   int(t.get("x_chunk", 0)), 1, int(t.get("granularity", 0)),
                   (ctypes.c_int32 * 2)(0, 0), 0.0)
    path = os.fsencode(cache) if cache else None
    ctx._rc(_lib.bem_autotune(ctx.h, ctypes.byref(op), len(entries), c, ctypes.byref(cfg), path,
                              _stream(stream)))
    return dict(grid=cfg.grid, tile_rows=cfg.tile_rows, tile_cols=cfg.tile_cols,
                x_chunk=cfg.x_chunk, granularity=cfg.granularity, tuned_ms=cfg.tuned_ms)


class Plan:
    """``bem_plan_batched``: one persistent, graph-captured assembly of many
    block lists.  ``entries`` is a list of (mesh, blocks, out, coupling)
    or (mesh, blocks, out, coupling, layers[, out2]) with layers one of
    BATCH_OP_LAYER (the operator's), BATCH_SLP, BATCH_DLP, BATCH_BOTH (near
    field, both layers in one pass: single layer to out, double layer to
    out2); the plan keeps references to them (the device pointers are
    captured).
    ``tune`` fixes fields of the launch configuration (grid, tile_rows,
    tile_cols, x_chunk); ``autotune`` times candidates for the others;
    ``cache`` names the tuning cache file."""

    def __init__(self, ctx, op, entries, tune=None, autotune=False, cache=None, stream=None):
        self.ctx, self.op, self.entries = ctx, op, list(entries)
        n = len(self.entries)
        self._c = (bem_batch * max(n, 1))()
        for k, e in enumerate(self.entries):
            self._c[k] = _batch(e)
        t = dict(tune or {})
        self.tune = bem_tune(int(t.get("grid", 0)), int(t.get("tile_rows", 0)),
                             int(t.get("tile_cols", 0)), int(t.get("x_chunk", 0)),
                             int(bool(autotune)), int(t.get("granularity", 0)),
                             (ctypes.c_int32 * 2)(0, 0), 0.0)
        h = ctypes.c_void_p()
        path = os.fsencode(cache) if cache else None
        ctx._rc(_lib.bem_plan_batched(ctx.h, ctypes.byref(op), n, self._c, ctypes.byref(self.tune),
                                      path, _stream(stream), ctypes.byref(h)))
        self.h = h

    @property
    def config(self):
        t = self.tune
        return dict(grid=t.grid, tile_rows=t.tile_rows, tile_cols=t.tile_cols,
                    x_chunk=t.x_chunk, granularity=t.granularity, tuned_ms=t.tuned_ms)

    @property
    def tiles(self):
        return int(_lib.bem_plan_tiles(self.h))

    def run(self, stream=None):
        self.ctx._rc(_lib.bem_run_batched(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            _lib.bem_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ learned form
def _setup_learned_api():
    P, i32, i64, f32, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                             ctypes.c_double)
    M, O, B = ctypes.POINTER(bem_mesh), ctypes.POINTER(bem_op), ctypes.POINTER(bem_blocks)
    _lib.bem_mlp_params.argtypes = [i32]
    _lib.bem_mlp_forward.argtypes = [P, i32, i32, P, i64, P, P, P]
    _lib.bem_mlp_grad.argtypes = [P, i32, P, i64, P, P, P, P, P]
    _lib.bem_mlp_adam.argtypes = [P, i64, P, P, P, P, i32, f32, f32, f32, f32, P]
    _lib.bem_selector_samples.argtypes = [P, M, O, i64, P, P, P, P, P]
    _lib.bem_select_orders.argtypes = [P, M, O, B, P, P, f64, f64, i32, i32, P, i64, P]
    _lib.bem_assemble_nearfield_learned.argtypes = [P, M, O, B, P, P, i64, P]
    _lib.bem_mlp_save.argtypes = [P, ctypes.c_char_p, i32, P, P, P, P, i32, P]
    _lib.bem_mlp_load.argtypes = [P, ctypes.c_char_p, i32, P, P, P, P, ctypes.POINTER(i32), P]
    _lib.bem_cluster_features.argtypes = [i32, P, P, P, P, f64, i32, f64, P]


_setup_learned_api()
SEL_OUT = 6  # selector outputs: predicted log10 error at orders 1 .. 6


def cluster_features(box, begin, end, height, kappa, side, eps):
    """bem_cluster_features: the rank head's eight inputs per cluster
    (float32 [n, 8]) from the cluster boxes, index ranges and heights."""
    import numpy as np
    box = np.ascontiguousarray(box, dtype=np.float64)
    begin = np.ascontiguousarray(begin, dtype=np.int32)
    end = np.ascontiguousarray(end, dtype=np.int32)
    height = np.ascontiguousarray(height, dtype=np.int32)
    n = begin.size
    if box.shape != (n, 6) or end.size != n or height.size != n:
        raise ValueError("box [n, 6], begin, end, height [n]")
    out = np.empty((n, 8), dtype=np.float32)
    rc = _lib.bem_cluster_features(n, _np_ptr(box), _np_ptr(begin), _np_ptr(end), _np_ptr(height),
                                   float(kappa), int(side), float(eps), _np_ptr(out))
    if rc != 0:
        raise BemError(rc, "bem_cluster_features: invalid arguments")
    return out


def mlp_params(n_out):
    n = _lib.bem_mlp_params(int(n_out))
    if n < 0:
        raise BemError(n, "n_out must be in [1, 16]")
    return n


def _context_mlp_forward(self, n_out, params, x, y, fp16=False, stream=None):
    self._rc(_lib.bem_mlp_forward(self.h, int(n_out), int(bool(fp16)), _ptr(params),
                                  x.shape[0], _ptr(x), _ptr(y), _stream(stream)))


def _context_mlp_grad(self, n_out, params, x, t, grad, loss=None, stream=None):
    self._rc(_lib.bem_mlp_grad(self.h, int(n_out), _ptr(params), x.shape[0], _ptr(x), _ptr(t),
                               _ptr(grad), _ptr(loss), _stream(stream)))


def _context_mlp_adam(self, params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                      stream=None):
    self._rc(_lib.bem_mlp_adam(self.h, params.numel(), _ptr(params), _ptr(grad), _ptr(m), _ptr(v),
                               int(step), float(lr), float(beta1), float(beta2), float(eps),
                               _stream(stream)))


def _context_selector_samples(self, mesh, op, rows, cols, x, t, stream=None):
    self._rc(_lib.bem_selector_samples(self.h, ctypes.byref(mesh.c), ctypes.byref(op),
                                       rows.numel(), _ptr(rows), _ptr(cols), _ptr(x), _ptr(t),
                                       _stream(stream)))


def _context_select_orders(self, mesh, op, blocks, params, orders, tol, margin, q_min=2,
                           stream=None, range=None, group=1):
    """bem_select_orders; range: device float[16] training range (or None);
    group: rows of a column sharing one decision (1: entry by entry)."""
    self._rc(_lib.bem_select_orders(self.h, ctypes.byref(mesh.c), ctypes.byref(op),
                                    ctypes.byref(blocks.c), _ptr(params), _ptr(range), float(tol),
                                    float(margin), int(q_min), int(group), _ptr(orders),
                                    orders.numel(), _stream(stream)))


def _context_assemble_nearfield_learned(self, mesh, op, blocks, orders, out, stream=None):
    self._rc(_lib.bem_assemble_nearfield_learned(self.h, ctypes.byref(mesh.c), ctypes.byref(op),
                                                 ctypes.byref(blocks.c), _ptr(orders), _ptr(out),
                                                 out.numel(), _stream(stream)))


def _context_mlp_save(self, path, n_out, params, m=None, v=None, range=None, step=0,
                      stream=None):
    """bem_mlp_save: network (and optionally Adam moments, training range)."""
    self._rc(_lib.bem_mlp_save(self.h, os.fsencode(path), int(n_out), _ptr(params), _ptr(m),
                               _ptr(v), _ptr(range), int(step), _stream(stream)))


def _context_mlp_load(self, path, n_out, params, m=None, v=None, range=None, stream=None):
    """bem_mlp_load into device tensors; returns the stored Adam step."""
    step = ctypes.c_int32()
    self._rc(_lib.bem_mlp_load(self.h, os.fsencode(path), int(n_out), _ptr(params), _ptr(m),
                               _ptr(v), _ptr(range), ctypes.byref(step), _stream(stream)))
    return step.value


Context.mlp_save = _context_mlp_save
Context.mlp_load = _context_mlp_load
Context.mlp_forward = _context_mlp_forward
Context.mlp_grad = _context_mlp_grad
Context.mlp_adam = _context_mlp_adam
Context.selector_samples = _context_selector_samples
Context.select_orders = _context_select_orders
Context.assemble_nearfield_learned = _context_assemble_nearfield_learned
