"""C ABI checks that need no GPU: the library loads, exports every function the
header declares, and rejects bad arguments before any HIP call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "irls_mincut.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(irls_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def P():
    import paper_1501_03105_amd as P
    P.lib()
    return P


def test_header_symbols_exported(P):
    names = declared_functions()
    assert "irls_mincut_create" in names and "irls_mincut_cut_batch" in names
    assert "irls_mincut_cut_two_level" in names
    lib = C.CDLL(P.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_options_layout(P):
    o = P.options()
    assert o.struct_size == C.sizeof(P.Options)
    assert o.rounds == 30 and o.eps0 == 0.1 and o.eps_factor == 0.5 and o.cg_rtol == 1e-10
    assert o.refine_every == 20 and o.fp64_weights_below_eps == 1e-4


def test_create_validation_errors(P):
    g = gen.gnp(10, 0.4, seed=2)
    E = P.create_error
    assert E(g.n, g.eu, g.ev, g.cap, 0, 0) == P.ERR_RANGE                     # s == t
    assert E(g.n, g.eu, g.ev, g.cap, 0, g.n) == P.ERR_RANGE                   # t out of range
    assert E(1, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0), 0, 1) == P.ERR_RANGE
    eu = g.eu.copy()
    eu[3] = g.n + 5
    assert E(g.n, eu, g.ev, g.cap, g.s, g.t) == P.ERR_RANGE
    for bad in (-1.0, 0.0, np.nan, np.inf):
        c = g.cap.copy()
        c[1] = bad
        assert E(g.n, g.eu, g.ev, c, g.s, g.t) == P.ERR_CAPACITY
    # a component touching neither s nor t
    assert E(6, np.array([0, 1, 3]), np.array([1, 5, 4]), np.ones(3), 0, 5) == P.ERR_DISCONNECTED
    # s and t in different components: rejected, G must be connected
    assert E(4, np.array([0, 2]), np.array([1, 3]), np.ones(2), 0, 3) == P.ERR_DISCONNECTED
    for kw in (dict(rounds=-1), dict(eps0=0.0), dict(eps_factor=1.5), dict(weight_form=2),
               dict(init=3), dict(cg_rtol=0.0), dict(cg_maxit=0), dict(precision=2),
               dict(format=3), dict(solver=3), dict(rows_per_wave=3), dict(rows_per_wave=128),
               dict(precision=1, solver=2), dict(struct_size=8), dict(unscaled_cg=2),
               dict(unscaled_cg=-1)):
        assert E(g.n, g.eu, g.ev, g.cap, g.s, g.t, **kw) == P.ERR_OPTIONS, kw
    # a graph that is not a grid cannot be forced into the diagonal format
    assert E(g.n, g.eu, g.ev, g.cap, g.s, g.t, format=2, solver=1) == P.ERR_OPTIONS


def test_null_handle_calls(P):
    L = P.lib()
    assert L.irls_mincut_solve(None, None, None) == P.ERR_NULL
    assert L.irls_mincut_cut(None, None, None, None) == P.ERR_NULL
    assert L.irls_mincut_cut_two_level(None, None, None, None) == P.ERR_NULL
    assert L.irls_mincut_update_capacities(None, 0, None, None, None) == P.ERR_NULL
    assert L.irls_mincut_cheeger_bracket(None, None, None) == P.ERR_NULL
    assert L.irls_mincut_set_row_lanes(None, None) == P.ERR_NULL
    assert L.irls_mincut_autotune(None, 1, 1, None) == P.ERR_NULL
    assert L.irls_mincut_potentials(None, None) == P.ERR_NULL
    L.irls_mincut_destroy(None)
    assert L.irls_mincut_last_error(None)
    h = C.c_void_p()
    assert L.irls_mincut_create(None, 3, 0, None, None, None, 0, 1, None, None) == P.ERR_NULL
    assert L.irls_mincut_create(C.byref(h), 4, 2, None, None, None, 0, 1, None, None) == P.ERR_NULL
    assert h.value is None
