"""Python view of the CPU oracle (ctypes over oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  Nothing on the product path may import it.
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_I64P = C.POINTER(C.c_int64)
_F64P = C.POINTER(C.c_double)
_U8P = C.POINTER(C.c_uint8)


class Options(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("eps0", C.c_double), ("eps_factor", C.c_double),
                ("weight_form", C.c_int32), ("init", C.c_int32), ("warm_start", C.c_int32),
                ("cg_rtol", C.c_double), ("cg_maxit", C.c_int64), ("threads", C.c_int32),
                ("precond", C.c_int32), ("block_size", C.c_int32)]


class Round(C.Structure):
    _fields_ = [("eps", C.c_double), ("cg_iters", C.c_int64), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("s_eps", C.c_double), ("l1", C.c_double),
                ("flow", C.c_double), ("flow_s", C.c_double), ("flow_t", C.c_double),
                ("vmin", C.c_double), ("vmax", C.c_double), ("status", C.c_int32),
                ("lower_bound", C.c_double)]


ROUND_FIELDS = [f for f, _ in Round._fields_]


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        G = [C.c_int64, C.c_int64, _I64P, _I64P, _F64P, C.c_int64, C.c_int64]
        L.orc_options_default.argtypes = [C.POINTER(Options)]
        L.orc_irls.argtypes = G + [C.POINTER(Options), _F64P, _F64P, C.POINTER(Round)]
        L.orc_irls_blocks.argtypes = G + [C.POINTER(Options), _I64P, _F64P, _F64P, C.POINTER(Round)]
        L.orc_reduced_system.argtypes = G + [_F64P, C.c_double, C.c_int32, _I64P, _I64P, _F64P, _F64P, _I64P]
        L.orc_sweep.argtypes = G + [_F64P, _U8P, _F64P, _I64P, C.POINTER(C.c_int32)]
        L.orc_block_apply.argtypes = G + [_F64P, C.c_double, C.c_int32, C.c_int32, C.c_int64, _I64P,
                                          _F64P, _F64P]
        L.orc_cut_value.argtypes = G + [_U8P, _F64P]
        L.orc_maxflow.argtypes = G + [_U8P, _F64P]
        L.orc_bruteforce.argtypes = G + [_U8P, _F64P, _F64P]
        L.orc_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t) if a is not None else None


def _graph_args(g):
    eu = np.ascontiguousarray(g.eu, dtype=np.int64)
    ev = np.ascontiguousarray(g.ev, dtype=np.int64)
    cap = np.ascontiguousarray(g.cap, dtype=np.float64)
    keep = (eu, ev, cap)
    return keep, [g.n, eu.shape[0], _p(eu, _I64P), _p(ev, _I64P), _p(cap, _F64P), g.s, g.t]


def options(**kw):
    o = Options()
    lib().orc_options_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def irls(g, x0=None, allow_maxit=False, block_of=None, **kw):
    """Run the oracle IRLS. Returns (x [n], list of per-round dicts, status).
    block_of: block id per node for the block-Jacobi preconditioner (precond
    1 exact, 2 ILU(0)); None: blocks of block_size consecutive rows."""
    o = options(**kw)
    keep, ga = _graph_args(g)
    x = np.zeros(g.n)
    rounds = (Round * (o.rounds + 1))()
    x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    ba = None if block_of is None else np.ascontiguousarray(block_of, dtype=np.int64)
    rc = lib().orc_irls_blocks(*ga, C.byref(o), _p(ba, _I64P), _p(x0a, _F64P), _p(x, _F64P), rounds)
    if rc not in (0, 100) or (rc == 100 and not allow_maxit):
        raise OracleError(rc, "irls")
    recs = [{f: getattr(r, f) for f in ROUND_FIELDS} for r in rounds]
    return x, recs, rc


def reduced_system(g, x=None, eps=0.0, weight_form=0):
    """Reduced Laplacian (CSR incl. diagonal) and right-hand side of one round."""
    keep, ga = _graph_args(g)
    nt = g.n - 2
    rowptr = np.zeros(nt + 1, np.int64)
    nnz = C.c_int64(0)
    xa = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
    rc = lib().orc_reduced_system(*ga, _p(xa, _F64P), eps, weight_form, _p(rowptr, _I64P),
                                  None, None, None, C.byref(nnz))
    if rc:
        raise OracleError(rc, "reduced_system")
    col = np.zeros(nnz.value, np.int64)
    val = np.zeros(nnz.value)
    b = np.zeros(nt)
    rc = lib().orc_reduced_system(*ga, _p(xa, _F64P), eps, weight_form, _p(rowptr, _I64P),
                                  _p(col, _I64P), _p(val, _F64P), _p(b, _F64P), C.byref(nnz))
    if rc:
        raise OracleError(rc, "reduced_system")
    return rowptr, col, val, b


def block_apply(g, r, kind, block_of=None, block_size=1, x=None, eps=0.0, weight_form=0):
    """z = M^-1 r for the block-Jacobi preconditioner of one round's system
    (kind 1 exact, 2 ILU(0)); r, z over the non-terminal nodes in ascending id."""
    keep, ga = _graph_args(g)
    ra = np.ascontiguousarray(r, dtype=np.float64)
    z = np.zeros(g.n - 2)
    xa = None if x is None else np.ascontiguousarray(x, dtype=np.float64)
    ba = None if block_of is None else np.ascontiguousarray(block_of, dtype=np.int64)
    rc = lib().orc_block_apply(*ga, _p(xa, _F64P), eps, weight_form, kind, block_size, _p(ba, _I64P),
                               _p(ra, _F64P), _p(z, _F64P))
    if rc:
        raise OracleError(rc, "block_apply")
    return z


def sweep(g, x):
    """Sweep cut of potentials x. Returns (in_S bool [n], value, kstar, scale)."""
    keep, ga = _graph_args(g)
    xa = np.ascontiguousarray(x, dtype=np.float64)
    inS = np.zeros(g.n, np.uint8)
    val = C.c_double(0)
    ks = C.c_int64(0)
    sc = C.c_int32(0)
    rc = lib().orc_sweep(*ga, _p(xa, _F64P), _p(inS, _U8P), C.byref(val), C.byref(ks), C.byref(sc))
    if rc:
        raise OracleError(rc, "sweep")
    return inS.astype(bool), val.value, ks.value, sc.value


def cut_value(g, in_S):
    keep, ga = _graph_args(g)
    a = np.ascontiguousarray(in_S, dtype=np.uint8)
    val = C.c_double(0)
    rc = lib().orc_cut_value(*ga, _p(a, _U8P), C.byref(val))
    if rc:
        raise OracleError(rc, "cut_value")
    return val.value


def maxflow(g):
    """Exact minimum cut by push-relabel. Returns (in_S bool [n], value)."""
    keep, ga = _graph_args(g)
    inS = np.zeros(g.n, np.uint8)
    val = C.c_double(0)
    rc = lib().orc_maxflow(*ga, _p(inS, _U8P), C.byref(val))
    if rc:
        raise OracleError(rc, "maxflow")
    return inS.astype(bool), val.value


def bruteforce(g):
    """Exhaustive minimum cut (n <= 24). Returns (in_S, value, second_value)."""
    keep, ga = _graph_args(g)
    inS = np.zeros(g.n, np.uint8)
    val = C.c_double(0)
    sec = C.c_double(0)
    rc = lib().orc_bruteforce(*ga, _p(inS, _U8P), C.byref(val), C.byref(sec))
    if rc:
        raise OracleError(rc, "bruteforce")
    return inS.astype(bool), val.value, sec.value


def max_threads():
    return lib().orc_max_threads()


def error_code(fn, *args, **kw):
    """Return the oracle's error code of a call (0 if it succeeds)."""
    try:
        fn(*args, **kw)
        return 0
    except OracleError as e:
        return e.code
