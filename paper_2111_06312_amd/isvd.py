"""ctypes binding of libisvd.so (argument marshalling only).

Every function here forwards device pointers of torch tensors, sizes and
the current HIP stream to the C ABI declared in include/isvd.h; all
arithmetic runs in the library's HIP kernels.  The library must have been
built (paper_2111_06312_amd/build.py); there is no fallback path.
"""

from __future__ import annotations

import ctypes as ct
import numbers
import os
from dataclasses import dataclass

import numpy as np
import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libisvd.so")
_lib = None

ISVD_OK, ISVD_E_INVALID, ISVD_E_OOM, ISVD_E_HIP, ISVD_E_NOT_SPD, ISVD_E_NOT_CONVERGED, ISVD_E_UNSUPPORTED = range(7)
FP64, FP32, BF16 = 0, 1, 2
FORM_NE, FORM_FEATPROP = 0, 1

_DTYPE = {FP64: torch.float64, FP32: torch.float32, BF16: torch.bfloat16}
_PREC = {torch.float64: FP64, torch.float32: FP32, torch.bfloat16: BF16}


class IsvdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"isvd status {status}: {msg}")
        self.status = status


class _Graph(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("nnz", ct.c_int64), ("indptr", ct.c_void_p), ("indices", ct.c_void_p),
                ("values", ct.c_void_p), ("symmetric", ct.c_int), ("t_indptr", ct.c_void_p),
                ("t_indices", ct.c_void_p), ("t_values", ct.c_void_p), ("add_self_loops", ct.c_int)]


class _Design(ct.Structure):
    _fields_ = [("form", ct.c_int), ("K", ct.c_int), ("coeffs", ct.POINTER(ct.c_double)), ("lam", ct.c_double),
                ("X", ct.c_void_p), ("d", ct.c_int64), ("ldx", ct.c_int64), ("L", ct.c_int)]


class _SvdParams(ct.Structure):
    _fields_ = [("k", ct.c_int), ("p", ct.c_int), ("q", ct.c_int), ("tol", ct.c_double), ("max_iter", ct.c_int),
                ("check_every", ct.c_int), ("seed", ct.c_uint64), ("omega", ct.c_void_p),
                ("ld_omega", ct.c_int64), ("fp32_switch_tol", ct.c_double), ("bf16_max_iter", ct.c_int),
                ("orth_passes", ct.c_int), ("orth_method", ct.c_int)]


class _SvdInfo(ct.Structure):
    _fields_ = [("iterations", ct.c_int), ("applies", ct.c_int), ("bf16_iterations", ct.c_int),
                ("residual_checks", ct.c_int), ("used_fallback", ct.c_int), ("residual", ct.c_double),
                ("seconds", ct.c_double), ("ritz_steps", ct.c_int), ("jacobi_sweeps", ct.c_int)]


@dataclass
class SvdInfo:
    iterations: int
    applies: int
    bf16_iterations: int
    residual_checks: int
    used_fallback: int
    residual: float
    seconds: float
    status: int = 0
    ritz_steps: int = 0
    jacobi_sweeps: int = 0


def load():
    """Load libisvd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2111_06312_amd/build.py")
    lib = ct.CDLL(_LIB_PATH)
    vp, i64, st = ct.c_void_p, ct.c_int64, ct.c_int
    lib.isvd_status_string.restype = ct.c_char_p
    lib.isvd_last_error.restype = ct.c_char_p
    lib.isvd_version.restype = ct.c_char_p
    lib.isvd_create_operator.argtypes = [ct.POINTER(_Graph), ct.POINTER(_Design), st, vp, ct.POINTER(vp)]
    lib.isvd_destroy_operator.argtypes = [vp]
    lib.isvd_destroy_operator.restype = None
    lib.isvd_operator_shape.argtypes = [vp, ct.POINTER(i64), ct.POINTER(i64)]
    lib.isvd_operator_gather_rows.argtypes = [vp, vp, i64, vp]
    lib.isvd_dag_create.argtypes = [st, ct.POINTER(vp)]
    lib.isvd_dag_destroy.argtypes = [vp]
    lib.isvd_dag_destroy.restype = None
    lib.isvd_dag_sparse.argtypes = [vp, i64, i64, i64, vp, vp, vp, st, vp, vp, vp, ct.POINTER(i64)]
    lib.isvd_dag_dense.argtypes = [vp, i64, i64, vp, i64, ct.POINTER(i64)]
    lib.isvd_dag_diag.argtypes = [vp, i64, vp, ct.POINTER(i64)]
    lib.isvd_dag_sum.argtypes = [vp, st, vp, vp, ct.POINTER(i64)]
    lib.isvd_dag_product.argtypes = [vp, st, vp, ct.POINTER(i64)]
    lib.isvd_dag_transpose.argtypes = [vp, i64, ct.POINTER(i64)]
    lib.isvd_dag_gather_rows.argtypes = [vp, i64, vp, i64, ct.POINTER(i64)]
    lib.isvd_dag_concat_cols.argtypes = [vp, st, vp, ct.POINTER(i64)]
    lib.isvd_dag_shape.argtypes = [vp, i64, ct.POINTER(i64), ct.POINTER(i64)]
    lib.isvd_dag_operator.argtypes = [vp, i64, st, ct.POINTER(vp)]
    lib.isvd_matmul_block.argtypes = [vp, st, vp, i64, i64, vp, i64, vp]
    lib.isvd_truncated_svd.argtypes = [vp, ct.POINTER(_SvdParams), vp, i64, vp, vp, i64, ct.POINTER(_SvdInfo), vp]
    lib.isvd_gaussian_block.argtypes = [i64, i64, ct.c_uint64, st, vp, i64, vp]
    lib.isvd_orthonormalize.argtypes = [i64, i64, st, vp, i64, vp, vp]
    lib.isvd_orthonormalize_householder.argtypes = [i64, i64, st, vp, i64, vp, vp]
    lib.isvd_gram.argtypes = [i64, i64, i64, st, vp, i64, vp, i64, vp, i64, vp]
    lib.isvd_gram_noalloc.argtypes = [i64, i64, i64, st, vp, i64, vp, i64, vp, i64, vp]
    lib.isvd_small_svd.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.isvd_ws_features.argtypes = [vp, vp, vp]
    lib.isvd_ws_create.argtypes = [st, ct.c_uint64, ct.POINTER(vp)]
    lib.isvd_ws_destroy.argtypes = [vp]
    lib.isvd_ws_destroy.restype = None
    lib.isvd_ws_num_params.argtypes = [vp]
    lib.isvd_ws_num_params.restype = i64
    lib.isvd_ws_get_params.argtypes = [vp, vp]
    lib.isvd_ws_set_params.argtypes = [vp, vp]
    lib.isvd_ws_forward.argtypes = [vp, i64, vp, vp, i64, vp]
    lib.isvd_ws_train_step.argtypes = [vp, i64, vp, vp, i64, ct.c_double, ct.POINTER(ct.c_double), vp, vp]
    lib.isvd_ws_omega.argtypes = [vp, vp, vp, st, ct.c_uint64, vp, i64, ct.POINTER(st), vp]
    lib.isvd_ne_embeddings.argtypes = [i64, i64, i64, st, vp, i64, vp, vp, i64, vp, i64, vp, i64, vp]
    lib.isvd_ne_scores.argtypes = [i64, st, vp, i64, i64, vp, vp, i64, i64, i64, vp, vp, vp, vp]
    lib.isvd_nc_fit.argtypes = [i64, i64, i64, i64, st, vp, i64, vp, vp, i64, vp, i64, vp, i64, ct.c_double,
                                vp, i64, vp]
    lib.isvd_profile_spmm_enable.argtypes = [st]
    lib.isvd_profile_learners_read.argtypes = [vp, vp, vp]
    lib.isvd_profile_spmm_read.argtypes = [ct.POINTER(ct.c_double), ct.POINTER(ct.c_double),
                                           ct.POINTER(ct.c_double), ct.POINTER(i64)]
    lib.isvd_peak_copy.argtypes = [vp, vp, i64, st, ct.POINTER(ct.c_double), vp]
    lib.isvd_peak_read.argtypes = [vp, i64, st, ct.POINTER(ct.c_double), vp]
    lib.isvd_peak_mfma.argtypes = [st, i64, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), vp]
    lib.isvd_profile_spmm_read_storage.argtypes = [st, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double),
                                                   ct.POINTER(ct.c_double), ct.POINTER(i64)]
    _lib = lib
    return lib


def _check(status, allow=()):
    if status != ISVD_OK and status not in allow:
        raise IsvdError(status, _lib.isvd_last_error().decode())
    return status


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _ld(t):
    assert t.dim() == 2 and t.stride(1) == 1, "blocks must be row-major with unit column stride"
    return t.stride(0)


class Operator:
    """Implicit design matrix on the GPU (isvd_create_operator).

    graph: an object with n, nnz, indptr (n+1 offsets) and indices (column
           ids) of the CSR of A, e.g. synth.Graph (host arrays are copied to
           the device and kept alive).
    form : "ne" (coeffs, lam, self_loops) or "featprop" (X torch tensor, L).
    values: edge weights of A in CSR order (None: every entry is 1).
    symmetric: A == A^T; otherwise t_indptr / t_indices (/ t_values, given
           exactly when values is) hold the CSR of A^T.
    """

    def __init__(self, graph, form="ne", coeffs=None, lam=0.0, self_loops=False, X=None, L=0,
                 precision=FP32, device="cuda", values=None, symmetric=True, t_indptr=None, t_indices=None,
                 t_values=None):
        lib = load()
        self.precision = precision
        self.dtype = _DTYPE[precision]
        self.n = graph.n

        def dev(a, dt, nonempty=False):
            if a is None:
                return None
            t = torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype=dt)), device=device)
            if nonempty and t.numel() == 0:
                t = torch.zeros(1, dtype=t.dtype, device=device)
            return t

        self._indptr = dev(graph.indptr, np.int64)
        self._indices = dev(graph.indices, np.int32, nonempty=True)
        self._values = dev(values, np.float32, nonempty=True)
        self._t_indptr = dev(t_indptr, np.int64)
        self._t_indices = dev(t_indices, np.int32, nonempty=True)
        self._t_values = dev(t_values, np.float32, nonempty=True)
        g = _Graph(n=graph.n, nnz=graph.nnz, indptr=self._indptr.data_ptr(), indices=self._indices.data_ptr(),
                   values=_ptr(self._values), symmetric=1 if symmetric else 0, t_indptr=_ptr(self._t_indptr),
                   t_indices=_ptr(self._t_indices), t_values=_ptr(self._t_values),
                   add_self_loops=1 if self_loops else 0)
        if form == "ne":
            c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
            self._coeffs = c
            dsn = _Design(form=FORM_NE, K=len(c), coeffs=c.ctypes.data_as(ct.POINTER(ct.c_double)),
                          lam=float(lam), X=None, d=0, ldx=0, L=0)
        elif form == "featprop":
            assert X is not None and X.dtype == self.dtype and X.is_cuda
            self._X = X
            dsn = _Design(form=FORM_FEATPROP, K=0, coeffs=None, lam=0.0, X=X.data_ptr(), d=X.shape[1],
                          ldx=_ld(X), L=int(L))
        else:
            raise ValueError(form)
        self.device = self._indptr.device
        handle = ct.c_void_p()
        _check(lib.isvd_create_operator(ct.byref(g), ct.byref(dsn), precision, _stream(), ct.byref(handle)))
        self.handle = handle
        r, cc = ct.c_int64(), ct.c_int64()
        _check(lib.isvd_operator_shape(handle, ct.byref(r), ct.byref(cc)))
        self.shape = (r.value, cc.value)

    def close(self):
        if getattr(self, "handle", None):
            _lib.isvd_destroy_operator(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def gather_rows(self, rows=None):
        """Restrict to M[rows, :] (distinct int64 indices; a device copy is
        taken) or, with rows=None, back to M (isvd_operator_gather_rows)."""
        try:
            if rows is None:
                _check(_lib.isvd_operator_gather_rows(self.handle, None, 0, _stream()))
            else:
                r = torch.as_tensor(rows, dtype=torch.int64, device=self.device).contiguous()
                _check(_lib.isvd_operator_gather_rows(self.handle, _ptr(r), r.shape[0], _stream()))
        finally:
            nr, nc = ct.c_int64(), ct.c_int64()
            _check(_lib.isvd_operator_shape(self.handle, ct.byref(nr), ct.byref(nc)))
            self.shape = (nr.value, nc.value)
        return self

    def matmul(self, Y, transpose=False, out=None):
        """M @ Y (or M^T @ Y) through isvd_matmul_block; enqueued on the current stream."""
        rows = self.shape[1] if transpose else self.shape[0]
        if out is None:
            out = torch.empty((rows, Y.shape[1]), dtype=self.dtype, device=Y.device)
        assert Y.dtype == self.dtype and out.dtype == self.dtype
        _check(_lib.isvd_matmul_block(self.handle, 1 if transpose else 0, _ptr(Y), _ld(Y), Y.shape[1],
                                      _ptr(out), _ld(out), _stream()))
        return out

    def truncated_svd(self, k, p, q=2, tol=0.0, max_iter=1000, check_every=0, seed=0, omega=None,
                      fp32_switch_tol=0.0, bf16_max_iter=0, orth_passes=0, allow_not_converged=False,
                      orth_method=0):
        """(U, S, V, info) through isvd_truncated_svd."""
        r, c = self.shape
        out_dtype = torch.float32 if self.precision == BF16 else self.dtype
        dev = self.device
        U = torch.empty((r, k), dtype=out_dtype, device=dev)
        V = torch.empty((c, k), dtype=out_dtype, device=dev)
        S = torch.empty(k, dtype=torch.float64, device=dev)
        prm = _SvdParams(k=k, p=p, q=q, tol=tol, max_iter=max_iter, check_every=check_every, seed=seed,
                         omega=_ptr(omega) if omega is not None else None,
                         ld_omega=_ld(omega) if omega is not None else 0, fp32_switch_tol=fp32_switch_tol,
                         bf16_max_iter=bf16_max_iter, orth_passes=orth_passes, orth_method=orth_method)
        if omega is not None:
            assert omega.dtype == self.dtype and omega.shape == (c, k + p)
        info = _SvdInfo()
        st = _check(_lib.isvd_truncated_svd(self.handle, ct.byref(prm), _ptr(U), k, _ptr(S), _ptr(V), k,
                                            ct.byref(info), _stream()),
                    allow=(ISVD_E_NOT_CONVERGED,) if allow_not_converged else ())
        return U, S, V, SvdInfo(info.iterations, info.applies, info.bf16_iterations, info.residual_checks,
                                info.used_fallback, info.residual, info.seconds, st, info.ritz_steps,
                                info.jacobi_sweeps)


class Dag:
    """A symbolic matrix DAG (isvd_dag_*): leaves hold device arrays, nodes
    combine them; `operator(node)` gives an Operator for products and the SVD.
    Leaf arrays are kept alive by this object."""

    def __init__(self, precision=FP32, device="cuda"):
        lib = load()
        assert precision in (FP32, FP64)
        self.precision = precision
        self.dtype = _DTYPE[precision]
        self.device = torch.device(device)
        self._keep = []
        h = ct.c_void_p()
        _check(lib.isvd_dag_create(precision, ct.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.isvd_dag_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _node(self, fn, *args):
        out = ct.c_int64()
        _check(fn(self.handle, *args, ct.byref(out)))
        return DagNode(self, out.value)

    def _ids(self, nodes):
        """Node ids as a C array; every node must belong to this DAG (an id
        is an index into one DAG's node store and means nothing in another)."""
        for nd in nodes:
            if not isinstance(nd, DagNode) or nd.dag is not self:
                raise ValueError("node belongs to another Dag")
        return (ct.c_int64 * len(nodes))(*[nd.id for nd in nodes])

    def sparse(self, indptr, indices, shape, values=None, symmetric=True, t_indptr=None, t_indices=None,
               t_values=None):
        """CSR leaf (host or device arrays; copied to the device and kept)."""
        def dev(a, dt):
            return None if a is None else torch.as_tensor(np.asarray(a) if not torch.is_tensor(a) else a,
                                                          dtype=dt, device=self.device).contiguous()
        arrs = [dev(indptr, torch.int64), dev(indices, torch.int32), dev(values, torch.float32),
                dev(t_indptr, torch.int64), dev(t_indices, torch.int32), dev(t_values, torch.float32)]
        for i in (1, 4):
            if arrs[i] is not None and arrs[i].numel() == 0:
                arrs[i] = torch.zeros(1, dtype=torch.int32, device=self.device)
        self._keep += [a for a in arrs if a is not None]
        nnz = int(arrs[0][-1].item())
        return self._node(_lib.isvd_dag_sparse, shape[0], shape[1], nnz, _ptr(arrs[0]), _ptr(arrs[1]),
                          _ptr(arrs[2]), 1 if symmetric else 0, _ptr(arrs[3]), _ptr(arrs[4]), _ptr(arrs[5]))

    def dense(self, X):
        assert X.dtype == self.dtype and X.is_cuda
        self._keep.append(X)
        return self._node(_lib.isvd_dag_dense, X.shape[0], X.shape[1], _ptr(X), _ld(X))

    def diag(self, d):
        t = torch.as_tensor(d, dtype=torch.float64, device=self.device).contiguous()
        return self._node(_lib.isvd_dag_diag, t.shape[0], _ptr(t))

    def sum(self, nodes, weights=None):
        ids = self._ids(nodes)
        w = None if weights is None else (ct.c_double * len(nodes))(*[float(x) for x in weights])
        return self._node(_lib.isvd_dag_sum, len(nodes), ids, w)

    def product(self, nodes):
        ids = self._ids(nodes)
        return self._node(_lib.isvd_dag_product, len(nodes), ids)

    def power(self, node, p):
        """node^p as a product of p references to node (p a positive integer)."""
        if isinstance(p, bool) or not isinstance(p, numbers.Integral) or p < 1:
            raise ValueError(f"matrix powers are positive integers, got {p!r}")
        factors = []
        for _ in range(int(p)):
            factors.append(node)
        return self.product(factors)

    def concat_cols(self, nodes):
        ids = self._ids(nodes)
        return self._node(_lib.isvd_dag_concat_cols, len(nodes), ids)

    def operator(self, node, lazy_cache=True):
        self._ids([node])
        h = ct.c_void_p()
        _check(_lib.isvd_dag_operator(self.handle, node.id, 1 if lazy_cache else 0, ct.byref(h)))
        op = Operator.__new__(Operator)
        op.precision = self.precision
        op.dtype = self.dtype
        op.device = self.device
        op.handle = h
        op._dag = self
        op.shape = node.shape
        op.n = node.shape[0]
        return op


class DagNode:
    """A node of a Dag; Python operators build new nodes (one C call each)."""

    def __init__(self, dag, nid):
        self.dag = dag
        self.id = nid
        r, c = ct.c_int64(), ct.c_int64()
        _check(_lib.isvd_dag_shape(dag.handle, nid, ct.byref(r), ct.byref(c)))
        self.shape = (r.value, c.value)

    @property
    def T(self):
        return self.dag._node(_lib.isvd_dag_transpose, self.id)

    def gather_rows(self, rows):
        r = torch.as_tensor(rows, dtype=torch.int64, device=self.dag.device).contiguous()
        return self.dag._node(_lib.isvd_dag_gather_rows, self.id, _ptr(r), r.shape[0])



def _same_dag_node(fn):
    def op(a, b):
        return fn(a, b) if isinstance(b, DagNode) else NotImplemented
    return op


def _scaled_node(a, s):
    return a.dag.sum([a], [float(s)]) if isinstance(s, numbers.Real) else NotImplemented


# a + b, a - b, s * a, a @ b and a ** p build DAG nodes (one C call each)
for _name, _fn in {
    "__add__": _same_dag_node(lambda a, b: a.dag.sum([a, b])),
    "__sub__": _same_dag_node(lambda a, b: a.dag.sum([a, b], [1.0, -1.0])),
    "__matmul__": _same_dag_node(lambda a, b: a.dag.product([a, b])),
    "__mul__": _scaled_node,
    "__rmul__": _scaled_node,
    "__pow__": lambda a, p: a.dag.power(a, p),
}.items():
    setattr(DagNode, _name, _fn)


def profile_spmm(on=True):
    """Start (or stop) event timing of every sparse pass."""
    load()
    _check(_lib.isvd_profile_spmm_enable(1 if on else 0))


def profile_spmm_read():
    """(total_ms, gather_bytes, compulsory_bytes, launches) since profile_spmm()."""
    ms, gb, cb, n = ct.c_double(), ct.c_double(), ct.c_double(), ct.c_int64()
    _check(_lib.isvd_profile_spmm_read(ct.byref(ms), ct.byref(gb), ct.byref(cb), ct.byref(n)))
    return ms.value, gb.value, cb.value, n.value


def profile_spmm_read_storage(precision):
    """(total_ms, gather_bytes, compulsory_bytes, launches) of the recorded
    passes over blocks stored in `precision` (FP64, FP32 or BF16); the
    record is kept for profile_spmm_read()."""
    ms, gb, cb, n = ct.c_double(), ct.c_double(), ct.c_double(), ct.c_int64()
    _check(_lib.isvd_profile_spmm_read_storage(precision, ct.byref(ms), ct.byref(gb), ct.byref(cb), ct.byref(n)))
    return ms.value, gb.value, cb.value, n.value


PHASES = ("products", "orthonormalisation", "rayleigh_ritz", "residual_checks", "output_products")


def profile_phases_read():
    """{phase: (ms, occurrences)} of the truncated SVDs since profiling was
    enabled or last read (event-timed on the SVD's stream); clears them."""
    load()
    ms = (ct.c_double * len(PHASES))()
    n = (ct.c_int64 * len(PHASES))()
    _check(_lib.isvd_profile_phases_read(ct.cast(ms, ct.c_void_p), ct.cast(n, ct.c_void_p)))
    return {name: (ms[i], n[i]) for i, name in enumerate(PHASES)}


def peak_copy(src, dst, reps=1):
    """Time `reps` device copies src -> dst (same byte size, 16-byte
    aligned) with the library's copy kernel; returns milliseconds."""
    load()
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nb
    ms = ct.c_double()
    _check(_lib.isvd_peak_copy(_ptr(src), _ptr(dst), nb, reps, ct.byref(ms), _stream()))
    return ms.value


def peak_read(src, reps=1):
    """Time one launch reading `src` `reps` times; returns milliseconds."""
    load()
    ms = ct.c_double()
    _check(_lib.isvd_peak_read(_ptr(src), src.numel() * src.element_size(), reps, ct.byref(ms), _stream()))
    return ms.value


def peak_mfma(precision, iters):
    """(flops, milliseconds) of back-to-back 16x16x4 MFMAs in FP64 or FP32."""
    load()
    fl, ms = ct.c_double(), ct.c_double()
    _check(_lib.isvd_peak_mfma(precision, iters, ct.byref(fl), ct.byref(ms), _stream()))
    return fl.value, ms.value


def profile_learners_read():
    """{name: (ms, algorithmic bytes, calls)} of the learner calls recorded
    since profile_spmm(True) or the last read."""
    ms = (ct.c_double * 3)()
    by = (ct.c_double * 3)()
    n = (ct.c_int64 * 3)()
    _check(_lib.isvd_profile_learners_read(ct.cast(ms, ct.c_void_p), ct.cast(by, ct.c_void_p),
                                           ct.cast(n, ct.c_void_p)))
    return {name: (ms[i], by[i], n[i]) for i, name in enumerate(("ne_embeddings", "ne_scores", "nc_fit"))}


def gaussian_block(rows, cols, seed, dtype=torch.float32, device="cuda"):
    load()
    out = torch.empty((rows, cols), dtype=dtype, device=device)
    _check(_lib.isvd_gaussian_block(rows, cols, seed, _PREC[dtype], _ptr(out), _ld(out), _stream()))
    return out


def orthonormalize(Y):
    """In place CholeskyQR2 of Y; returns (Y, R) with R an FP64 tensor."""
    load()
    l = Y.shape[1]
    R = torch.empty((l, l), dtype=torch.float64, device=Y.device)
    _check(_lib.isvd_orthonormalize(Y.shape[0], l, _PREC[Y.dtype], _ptr(Y), _ld(Y), _ptr(R), _stream()))
    return Y, R


def orthonormalize_householder(Y):
    """In place Householder QR of Y; returns (Y, R) with R an FP64 tensor."""
    load()
    l = Y.shape[1]
    R = torch.empty((l, l), dtype=torch.float64, device=Y.device)
    _check(_lib.isvd_orthonormalize_householder(Y.shape[0], l, _PREC[Y.dtype], _ptr(Y), _ld(Y), _ptr(R), _stream()))
    return Y, R


def gram(A, B=None):
    """A^T B in FP64 (B defaults to A)."""
    load()
    B = A if B is None else B
    C = torch.empty((A.shape[1], B.shape[1]), dtype=torch.float64, device=A.device)
    _check(_lib.isvd_gram(A.shape[0], A.shape[1], B.shape[1], _PREC[A.dtype], _ptr(A), _ld(A), _ptr(B), _ld(B),
                          _ptr(C), C.shape[1], _stream()))
    return C


def gram_noalloc(A, B, C):
    """C <- A^T B in FP64 through isvd_gram_noalloc (no allocation by the
    library; C is the caller's m x p FP64 tensor); enqueued on the current
    stream."""
    load()
    assert C.dtype == torch.float64 and C.shape == (A.shape[1], B.shape[1])
    _check(_lib.isvd_gram_noalloc(A.shape[0], A.shape[1], B.shape[1], _PREC[A.dtype], _ptr(A), _ld(A), _ptr(B),
                                  _ld(B), _ptr(C), _ld(C), _stream()))
    return C


def small_svd(A):
    """(U, s, V) of a small square FP64 matrix by one-sided Jacobi."""
    load()
    n = A.shape[0]
    A = A.contiguous()
    U = torch.empty_like(A)
    V = torch.empty_like(A)
    s = torch.empty(n, dtype=torch.float64, device=A.device)
    _check(_lib.isvd_small_svd(n, _ptr(A), _ptr(U), _ptr(s), _ptr(V), _stream()))
    return U, s, V


def _factor_prec(U, S, V):
    assert U.dtype == V.dtype and U.dtype in (torch.float32, torch.float64), "U and V must be FP32 or FP64"
    assert U.shape[1] == V.shape[1], "U and V need the same rank"
    assert S.dtype == torch.float64 and S.is_contiguous() and S.shape[0] == U.shape[1], "S: k FP64 values"
    return _PREC[U.dtype]


def ne_embeddings(U, S, V):
    """(L, R) = (U S^(1/2), V S^(1/2)) of Eq. 5, in the precision of U and V."""
    load()
    prec = _factor_prec(U, S, V)
    k = U.shape[1]
    L = torch.empty_like(U, memory_format=torch.contiguous_format)
    R = torch.empty_like(V, memory_format=torch.contiguous_format)
    _check(_lib.isvd_ne_embeddings(U.shape[0], V.shape[0], k, prec, _ptr(U), _ld(U), _ptr(S), _ptr(V), _ld(V),
                                   _ptr(L), k, _ptr(R), k, _stream()))
    return L, R


def ne_scores(U, S, V, pi, pj):
    """FP64 scores U[i] S V[j]^T (Eq. 5) of the pairs (pi[p], pj[p]) (int64 device tensors)."""
    load()
    prec = _factor_prec(U, S, V)
    pi = pi.to(torch.int64).contiguous()
    pj = pj.to(torch.int64).contiguous()
    assert pi.shape == pj.shape and pi.dim() == 1
    out = torch.empty(pi.shape[0], dtype=torch.float64, device=U.device)
    _check(_lib.isvd_ne_scores(U.shape[1], prec, _ptr(U), _ld(U), U.shape[0], _ptr(S), _ptr(V), _ld(V), V.shape[0],
                               pi.shape[0], _ptr(pi), _ptr(pj), _ptr(out), _stream()))
    return out


def nc_fit(U, S, V, Y, rows=None, rcond=0.0):
    """Least-norm W = V S^+ U^T Y of Eq. 8 (FP64, V.shape[0] x Y.shape[1]).

    Y has the dtype of U; rows (int64 device tensor) keeps only those rows of
    U and Y (the labelled nodes)."""
    load()
    prec = _factor_prec(U, S, V)
    assert Y.dtype == U.dtype and Y.shape[0] == U.shape[0]
    ny = Y.shape[1]
    W = torch.empty((V.shape[0], ny), dtype=torch.float64, device=U.device)
    if rows is not None:
        rows = rows.to(torch.int64).contiguous()
    _check(_lib.isvd_nc_fit(U.shape[0], V.shape[0], U.shape[1], ny, prec, _ptr(U), _ld(U), _ptr(S), _ptr(V), _ld(V),
                            _ptr(Y), _ld(Y), _ptr(rows), -1 if rows is None else rows.shape[0], float(rcond),
                            _ptr(W), ny, _stream()))
    return W


def exported_symbols_from_header(path=None):
    """Names of the functions include/isvd.h declares (for the export test)."""
    import re
    path = path or os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "isvd.h")
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(isvd_[a-z0-9_]+)\s*\(", text)))


def features(op):
    """n x 16 FP32 structural features of an NE operator's nodes (isvd_ws_features)."""
    load()
    F = torch.empty((op.shape[1], 16), dtype=torch.float32, device=op._indptr.device)
    _check(_lib.isvd_ws_features(op.handle, _ptr(F), _stream()))
    return F


class WarmStart:
    """The warm-start network (isvd_ws_*): 16 -> 128 -> 128 -> k MLP."""

    def __init__(self, k, seed=0):
        load()
        h = ct.c_void_p()
        _check(_lib.isvd_ws_create(k, seed, ct.byref(h)))
        self.handle = h
        self.k = k

    def close(self):
        if getattr(self, "handle", None):
            _lib.isvd_ws_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self):
        return _lib.isvd_ws_num_params(self.handle)

    def get_params(self):
        out = np.empty(self.num_params, dtype=np.float32)
        _check(_lib.isvd_ws_get_params(self.handle, out.ctypes.data_as(ct.c_void_p)))
        return out

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == self.num_params
        _check(_lib.isvd_ws_set_params(self.handle, theta.ctypes.data_as(ct.c_void_p)))

    def forward(self, F):
        Z = torch.empty((F.shape[0], self.k), dtype=torch.float32, device=F.device)
        _check(_lib.isvd_ws_forward(self.handle, F.shape[0], _ptr(F), _ptr(Z), self.k, _stream()))
        return Z

    def train_step(self, F, V, lr=0.0, want_grad=False):
        """(loss, grad or None); applies an Adam step when lr > 0."""
        loss = ct.c_double()
        grad = np.empty(self.num_params, dtype=np.float32) if want_grad else None
        _check(_lib.isvd_ws_train_step(self.handle, F.shape[0], _ptr(F), _ptr(V), _ld(V), float(lr), ct.byref(loss),
                                       grad.ctypes.data_as(ct.c_void_p) if want_grad else None, _stream()))
        return loss.value, grad

    def omega(self, op, F, p, seed=0):
        """(start block [MLP(F) | Gaussian p columns] in op's precision, used_fallback)."""
        c = op.shape[1]
        om = torch.empty((c, self.k + p), dtype=op.dtype, device=F.device)
        fb = ct.c_int()
        _check(_lib.isvd_ws_omega(self.handle, op.handle, _ptr(F), p, seed, _ptr(om), _ld(om), ct.byref(fb),
                                  _stream()))
        return om, bool(fb.value)
