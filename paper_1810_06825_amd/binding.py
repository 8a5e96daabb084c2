"""ctypes binding of the C interface in include/frpca.h (argument marshalling only).

Every function here forwards to the entry point of the same name in the in-tree HIP
library _lib/libfrpca.so; a non-zero status becomes FrpcaError carrying the library's
message. There is no fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libfrpca.so")

FRPCA_OK = 0
FRPCA_EINVAL = -1
FRPCA_ENOMEM = -2
FRPCA_EHIP = -3
FRPCA_ESTATE = -4
NTIMERS = 15
TIMER_NAMES = ("gauss", "spmm_fwd", "spmm_back", "gram", "eig", "lu", "tsmm", "sign", "bwd", "sddmm",
               "spmm_fixup", "spmm_combine",
               "spmm_back_tail", "center", "qr")


class FrpcaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"frpca error {code}: {msg}")
        self.code = code


class FrpcaOpts(ctypes.Structure):
    _fields_ = [("panel_bf16", c_int), ("no_sign_fix", c_int), ("rank_tol", c_double),
                ("timing", c_int), ("max_workspace", c_size_t), ("center", c_int),
                ("gram_f32", c_int), ("fused_pass", c_int), ("final_f64", c_int)]


class FrpcaInfo(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("nnz", c_int64), ("orientation", c_int),
                ("k", c_int), ("s", c_int), ("passes", c_int), ("rank_dropped", c_int),
                ("workspace_bytes", c_size_t), ("create_ms", c_double), ("hot_cols", c_int64),
                ("row_blocks", c_int64), ("hot_nnz", c_int64),
                ("t_ms", c_double * NTIMERS), ("t_count", c_int64 * NTIMERS)]


_SIGNATURES = {
    "frpca_create": (c_int, [POINTER(c_void_p), c_int64, c_int64, c_int64, c_void_p, c_void_p, c_void_p,
                             POINTER(FrpcaOpts), c_void_p]),
    "frpca_set_values": (c_int, [c_void_p, c_void_p]),
    "frpca_set_stream": (c_int, [c_void_p, c_void_p]),
    "frpca_run": (c_int, [c_void_p, c_int, c_int, c_int, c_uint64, c_void_p, c_void_p, c_void_p]),
    "frpca_run_basic": (c_int, [c_void_p, c_int, c_int, c_int, c_uint64, c_int, c_void_p, c_void_p, c_void_p]),
    "frpca_eigsvds": (c_int, [c_void_p, c_int, c_int, c_uint64, c_double, c_int, c_void_p, c_void_p, c_void_p,
                              POINTER(c_int)]),
    "frpca_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "frpca_adjoint": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                              c_void_p]),
    "frpca_get_info": (c_int, [c_void_p, POINTER(FrpcaInfo)]),
    "frpca_reset_timers": (c_int, [c_void_p]),
    "frpca_last_error": (c_char_p, [c_void_p]),
    "frpca_destroy": (c_int, [c_void_p]),
    "frpca_gaussian": (c_int, [c_void_p, c_uint64, c_int64, c_int, c_int, c_void_p]),
    "frpca_spmm": (c_int, [c_void_p, c_int, c_int, c_void_p, c_int, c_int, c_void_p, c_int, c_int]),
    "frpca_gram": (c_int, [c_void_p, c_int64, c_int, c_void_p, c_int, c_void_p]),
    "frpca_eig": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "frpca_eig_noalloc": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "frpca_eigsvd": (c_int, [c_void_p, c_int64, c_int, c_void_p, c_int, c_void_p, c_int, c_void_p, c_double]),
    "frpca_lu": (c_int, [c_void_p, c_int64, c_int, c_void_p, c_int, c_void_p, c_int, c_double, POINTER(c_int)]),
    "frpca_orth": (c_int, [c_void_p, c_int64, c_int, c_void_p, c_int, c_void_p, c_int, c_void_p, POINTER(c_int)]),
    "frpca_jacobi_svd": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "frpca_pass": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int]),
    "frpca_tsmm": (c_int, [c_void_p, c_int64, c_int, c_int, c_void_p, c_int, c_void_p, c_void_p, c_int]),
    "frpca_sddmm": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "frpca_gather_probe": (c_int, [c_void_p, c_void_p, c_int64, c_int, c_int64, c_uint32, c_void_p,
                                   POINTER(c_float), POINTER(c_int64)]),
    "frpca_export_csc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
}

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def exported_symbols() -> list:
    return list(_SIGNATURES)


def _check(rc: int, h=None) -> None:
    if rc != FRPCA_OK:
        msg = load().frpca_last_error(h)
        raise FrpcaError(rc, msg.decode() if msg else "")


def _ptr(t):
    """Device (or host) address of a tensor / int / None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


# ------------------------------------------------------------------ same-name wrappers
def frpca_create(m, n, nnz, row_ptr, col, val, opts=None, stream=None):
    h = c_void_p()
    o = opts if opts is not None else FrpcaOpts()
    _check(load().frpca_create(ctypes.byref(h), m, n, nnz, _ptr(row_ptr), _ptr(col), _ptr(val), ctypes.byref(o),
                               stream))
    return h


def frpca_set_values(h, val):
    _check(load().frpca_set_values(h, _ptr(val)), h)


def frpca_set_stream(h, stream):
    _check(load().frpca_set_stream(h, stream), h)


def frpca_run(h, k, p_passes, s_oversample, seed, U, S, V):
    _check(load().frpca_run(h, k, p_passes, s_oversample, seed, _ptr(U), _ptr(S), _ptr(V)), h)


def frpca_run_basic(h, k, p_power, s_oversample, seed, alg, U, S, V):
    _check(load().frpca_run_basic(h, k, p_power, s_oversample, seed, alg, _ptr(U), _ptr(S), _ptr(V)), h)


def frpca_eigsvds(h, k, s_oversample, seed, tol, max_iter, U, S, V) -> int:
    it = c_int(0)
    _check(load().frpca_eigsvds(h, k, s_oversample, seed, tol, max_iter, _ptr(U), _ptr(S), _ptr(V), ctypes.byref(it)),
           h)
    return it.value


def frpca_backward(h, dU, dS, dV, dval):
    _check(load().frpca_backward(h, _ptr(dU), _ptr(dS), _ptr(dV), _ptr(dval)), h)


def frpca_adjoint(h, k, U, S, V, dU, dS, dV, dval):
    _check(load().frpca_adjoint(h, k, _ptr(U), _ptr(S), _ptr(V), _ptr(dU), _ptr(dS), _ptr(dV), _ptr(dval)), h)


def frpca_get_info(h) -> FrpcaInfo:
    info = FrpcaInfo()
    _check(load().frpca_get_info(h, ctypes.byref(info)), h)
    return info


def frpca_reset_timers(h):
    _check(load().frpca_reset_timers(h), h)


def frpca_last_error(h=None) -> str:
    msg = load().frpca_last_error(h)
    return msg.decode() if msg else ""


def frpca_destroy(h):
    _check(load().frpca_destroy(h))


def frpca_gaussian(h, seed, rows, l, ld, out):
    _check(load().frpca_gaussian(h, seed, rows, l, ld, _ptr(out)), h)


def frpca_spmm(h, trans, l, inp, in_bf16, ld_in, out, out_bf16, ld_out):
    _check(load().frpca_spmm(h, trans, l, _ptr(inp), in_bf16, ld_in, _ptr(out), out_bf16, ld_out), h)


def frpca_gram(h, rows, l, X, ldx, G):
    _check(load().frpca_gram(h, rows, l, _ptr(X), ldx, _ptr(G)), h)


def frpca_eig(h, l, G, W, d):
    _check(load().frpca_eig(h, l, _ptr(G), _ptr(W), _ptr(d)), h)


def frpca_eig_noalloc(l, G, W, d, stream=None):
    _check(load().frpca_eig_noalloc(l, _ptr(G), _ptr(W), _ptr(d), stream))


def frpca_eigsvd(h, rows, l, X, ldx, Q, ldq, S, tol=0.0):
    _check(load().frpca_eigsvd(h, rows, l, _ptr(X), ldx, _ptr(Q), ldq, _ptr(S), tol), h)


def frpca_lu(h, rows, l, X, ldx, Q, ldq, tol=0.0) -> int:
    nd = c_int(0)
    _check(load().frpca_lu(h, rows, l, _ptr(X), ldx, _ptr(Q), ldq, tol, ctypes.byref(nd)), h)
    return nd.value


def frpca_orth(h, rows, l, X, ldx, Q, ldq, R=None) -> int:
    nd = c_int(0)
    _check(load().frpca_orth(h, rows, l, _ptr(X), ldx, _ptr(Q), ldq, _ptr(R), ctypes.byref(nd)), h)
    return nd.value


def frpca_jacobi_svd(h, l, R, W, d):
    _check(load().frpca_jacobi_svd(h, l, _ptr(R), _ptr(W), _ptr(d)), h)


def frpca_pass(h, l, inp, out, fused):
    _check(load().frpca_pass(h, l, _ptr(inp), _ptr(out), fused), h)


def frpca_tsmm(h, rows, kdim, c, X, ldx, B, out, ldo):
    _check(load().frpca_tsmm(h, rows, kdim, c, _ptr(X), ldx, _ptr(B), _ptr(out), ldo), h)


def frpca_gather_probe(h, P, rows, ld, gathers, seed, out):
    """Random 512-byte row reads of P; returns (ms, rows_read)."""
    ms, nr = c_float(0.0), c_int64(0)
    _check(load().frpca_gather_probe(h, _ptr(P), rows, ld, gathers, seed, _ptr(out), ctypes.byref(ms),
                                     ctypes.byref(nr)), h)
    return ms.value, nr.value


def frpca_sddmm(h, w, P1, Q1, P2, Q2, dval):
    _check(load().frpca_sddmm(h, w, _ptr(P1), _ptr(Q1), _ptr(P2), _ptr(Q2), _ptr(dval)), h)


def frpca_export_csc(h, col_ptr, row, perm):
    _check(load().frpca_export_csc(h, _ptr(col_ptr), _ptr(row), _ptr(perm)), h)
