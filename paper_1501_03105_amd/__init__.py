"""Python binding of libirls_mincut, the MI355X IRLS s-t min-cut library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  The names follow the C ABI in include/irls_mincut.h.  Arrays may
be numpy arrays (host) or torch CUDA tensors (device; the options then set
inputs_on_device).  Importing this module raises if the HIP library has not
been built: there is no CPU fallback.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libirls_mincut.so")

OK, ERR_NULL, ERR_RANGE, ERR_CAPACITY, ERR_DISCONNECTED, ERR_OPTIONS = 0, 1, 2, 3, 4, 5
ERR_NOT_SOLVED, ERR_CG_BREAKDOWN, ERR_DEVICE, ERR_OOM, WARN_CG_MAXIT = 6, 7, 8, 9, 100


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_int32), ("rounds", C.c_int32), ("eps0", C.c_double),
                ("eps_factor", C.c_double), ("weight_form", C.c_int32), ("init", C.c_int32),
                ("warm_start", C.c_int32), ("cg_rtol", C.c_double), ("cg_maxit", C.c_int64),
                ("precision", C.c_int32), ("refine_every", C.c_int32),
                ("fp64_weights_below_eps", C.c_double), ("format", C.c_int32),
                ("solver", C.c_int32), ("chunk", C.c_int32), ("inputs_on_device", C.c_int32),
                ("rows_per_wave", C.c_int32), ("precond", C.c_int32), ("block_size", C.c_int32),
                ("unscaled_cg", C.c_int32), ("stop_gap", C.c_double)]


class RoundStats(C.Structure):
    _fields_ = [("eps", C.c_double), ("cg_iters", C.c_int64), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double), ("s_eps", C.c_double), ("l1", C.c_double),
                ("flow", C.c_double), ("flow_s", C.c_double), ("flow_t", C.c_double),
                ("vmin", C.c_double), ("vmax", C.c_double), ("status", C.c_int32),
                ("lower_bound", C.c_double)]


STAT_FIELDS = [f for f, _ in RoundStats._fields_]


class TwoLevelInfo(C.Structure):
    _fields_ = [("c0", C.c_double), ("c1", C.c_double), ("gamma0", C.c_double), ("gamma1", C.c_double),
                ("kmeans_updates", C.c_int32), ("n_s0", C.c_int64), ("n_s1", C.c_int64),
                ("n_sc", C.c_int64), ("coarse_edges", C.c_int64), ("coarse_value", C.c_double)]


class IrlsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"irls_mincut error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libirls_mincut.so; raises if it is missing (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1501_03105_amd/build.py")
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        P64, PF64, PU8 = C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_uint8)
        L.irls_options_default.argtypes = [C.POINTER(Options)]
        L.irls_options_default.restype = None
        L.irls_mincut_create.argtypes = [C.POINTER(H), C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                         C.c_void_p, C.c_int64, C.c_int64, C.POINTER(Options), C.c_void_p]
        L.irls_mincut_solve.argtypes = [H, C.c_void_p, C.POINTER(RoundStats)]
        L.irls_mincut_solve_range.argtypes = [H, C.c_int32, C.c_void_p, C.c_double, C.c_int32,
                                              C.POINTER(RoundStats)]
        L.irls_mincut_cut.argtypes = [H, PU8, PF64, P64]
        L.irls_mincut_cut_noalloc.argtypes = [H, PU8, PF64, P64]
        L.irls_mincut_cut_two_level.argtypes = [H, PU8, PF64, C.POINTER(TwoLevelInfo)]
        L.irls_mincut_update_capacities.argtypes = [H, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.irls_mincut_cheeger_bracket.argtypes = [H, PF64, PF64]
        L.irls_mincut_potentials.argtypes = [H, PF64]
        L.irls_mincut_set_potentials.argtypes = [H, C.c_void_p]
        L.irls_mincut_info.argtypes = [H, P64, P64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.irls_mincut_time_kernel.argtypes = [H, C.c_int32, C.c_int32, PF64]
        L.irls_mincut_spmv_kernel.argtypes = [H, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.irls_mincut_set_kernel_timing.argtypes = [H, C.c_int32, C.c_int32]
        L.irls_mincut_set_march_tile.argtypes = [H, C.c_int32, C.c_int32]
        L.irls_stream_probe.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                        PF64]
        L.irls_stream_probe.restype = C.c_int
        L.irls_mincut_march_tile.argtypes = [H, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                             C.POINTER(C.c_int32)]
        L.irls_mincut_kernel_timing.argtypes = [H, PF64, P64, PF64, P64]
        L.irls_mincut_destroy.argtypes = [H]
        L.irls_mincut_destroy.restype = None
        L.irls_mincut_last_error.argtypes = [H]
        L.irls_mincut_last_error.restype = C.c_char_p
        L.irls_mincut_create_batch.argtypes = [C.POINTER(H), C.c_int32, P64, P64, P64, P64, PF64,
                                               P64, P64, C.POINTER(Options), C.c_void_p]
        L.irls_mincut_solve_batch.argtypes = [H, C.POINTER(RoundStats)]
        L.irls_mincut_cut_batch.argtypes = [H, PU8, PF64]
        P32 = C.POINTER(C.c_int32)
        L.irls_mincut_set_row_lanes.argtypes = [H, P32]
        L.irls_mincut_autotune.argtypes = [H, C.c_int32, C.c_int32, P32]
        for f in ("create", "solve", "solve_range", "cut", "cut_noalloc", "cut_two_level", "update_capacities",
                  "cheeger_bracket", "potentials",
                  "set_potentials",
                  "info", "time_kernel", "spmv_kernel", "set_kernel_timing", "kernel_timing",
                  "set_march_tile", "march_tile",
                  "create_batch", "solve_batch", "cut_batch",
                  "set_row_lanes", "autotune"):
            getattr(L, "irls_mincut_" + f).restype = C.c_int
        PF32 = C.POINTER(C.c_float)
        L.irls_gnn_create.argtypes = [C.POINTER(H), C.c_int32, C.c_int32, C.c_uint64, C.c_void_p]
        L.irls_gnn_num_params.argtypes = [H, P64]
        L.irls_gnn_get_params.argtypes = [H, PF32]
        L.irls_gnn_set_params.argtypes = [H, PF32]
        L.irls_gnn_predict.argtypes = [H, H, PF64, PF64, PF64, PF64]
        L.irls_gnn_warm_start.argtypes = [H, H, PF64, C.c_double, PF64]
        L.irls_gnn_loss_grad.argtypes = [H, H, PF64, PF64, PF64, C.c_double, C.c_double, PF64, PF32]
        L.irls_gnn_adam_step.argtypes = [H, C.c_double, C.c_double, C.c_double, C.c_double]
        L.irls_gnn_destroy.argtypes = [H]
        L.irls_gnn_destroy.restype = None
        L.irls_gnn_last_error.argtypes = [H]
        L.irls_gnn_last_error.restype = C.c_char_p
        for f in ("create", "num_params", "get_params", "set_params", "predict", "warm_start", "loss_grad",
                  "adam_step"):
            getattr(L, "irls_gnn_" + f).restype = C.c_int
        o = Options()
        L.irls_options_default(C.byref(o))
        if o.struct_size != C.sizeof(Options):
            raise ImportError("irls_options layout mismatch between binding and library")
        _lib = L
    return _lib


def options(**kw):
    o = Options()
    lib().irls_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a, dtype):
    """Device/host address of a contiguous array; returns (ptr, keepalive, on_device)."""
    if a is None:
        return None, None, False
    if _is_torch(a):
        import torch
        tdt = {np.int64: torch.int64, np.float64: torch.float64}[dtype]
        t = a.to(tdt).contiguous()
        return t.data_ptr(), t, t.is_cuda
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, arr, False


def _ptr_as(a, dtype, on_device):
    """_ptr with the array moved where the handle reads its inputs: a CUDA
    tensor for a handle created with inputs_on_device, host memory otherwise."""
    if a is None:
        return None, None, False
    if on_device:
        import torch
        tdt = {np.int64: torch.int64, np.float64: torch.float64}[dtype]
        t = (a if _is_torch(a) else torch.as_tensor(np.asarray(a))).to(device="cuda", dtype=tdt).contiguous()
        return t.data_ptr(), t, True
    if _is_torch(a):
        a = a.detach().cpu().numpy()
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data, arr, False


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream        # torch.cuda.Stream


def _stats_list(arr):
    return [{f: getattr(r, f) for f in STAT_FIELDS} for r in arr]


ROW_LANE_BINS = 6


class _RowLanes:
    """Rows per wavefront of the resident solver (irls_mincut_set_row_lanes,
    irls_mincut_autotune); lanes[b] = lanes per row of length bin b."""

    def set_row_lanes(self, lanes):
        arr = (C.c_int32 * ROW_LANE_BINS)(*[int(x) for x in lanes])
        rc = lib().irls_mincut_set_row_lanes(self.h, arr)
        if rc != OK:
            raise self._err(rc)

    def autotune(self, rounds=1, reps=2):
        """Times candidate tables and keeps the fastest; returns it."""
        arr = (C.c_int32 * ROW_LANE_BINS)()
        rc = lib().irls_mincut_autotune(self.h, rounds, reps, arr)
        if rc != OK:
            raise self._err(rc)
        return list(arr)


class MinCut(_RowLanes):
    """One graph on the GPU: irls_mincut_create / _solve / _cut / ... / _destroy."""

    def __init__(self, n, eu, ev, cap, s, t, stream=None, **opts):
        L = lib()
        pu, ku, du = _ptr(eu, np.int64)
        pv, kv, dv = _ptr(ev, np.int64)
        pc, kc, dc = _ptr(cap, np.float64)
        if opts.get("inputs_on_device") is None and (du or dv or dc):
            opts["inputs_on_device"] = 1
        self.opt = options(**opts)
        self.n, self.s, self.t = int(n), int(s), int(t)
        m = 0 if ku is None else int(ku.shape[0] if hasattr(ku, "shape") else len(ku))
        h = C.c_void_p()
        rc = L.irls_mincut_create(C.byref(h), self.n, m, pu, pv, pc, self.s, self.t,
                                  C.byref(self.opt), _stream_ptr(stream))
        if rc != OK:
            raise IrlsError(rc, L.irls_mincut_last_error(None).decode())
        self.h = h

    @classmethod
    def from_graph(cls, g, **kw):
        return cls(g.n, g.eu, g.ev, g.cap, g.s, g.t, **kw)

    def _err(self, rc):
        return IrlsError(rc, lib().irls_mincut_last_error(self.h).decode())

    def solve(self, x0=None, allow_maxit=True):
        """Run all rounds. Returns (status, per-round stats list)."""
        st = (RoundStats * (self.opt.rounds + 1))()
        px, keep, _ = _ptr_as(x0, np.float64, self.opt.inputs_on_device)
        rc = lib().irls_mincut_solve(self.h, px, st)
        if rc not in (OK, WARN_CG_MAXIT) or (rc == WARN_CG_MAXIT and not allow_maxit):
            raise self._err(rc)
        return rc, _stats_list(st)

    def solve_range(self, start, rounds, eps_first=-1.0, x0=None):
        """irls_mincut_solve_range: start 0 (options), 1 (continue), 2 (from x0)."""
        st = (RoundStats * (rounds + 1))()
        px, keep, _ = _ptr_as(x0, np.float64, self.opt.inputs_on_device)
        rc = lib().irls_mincut_solve_range(self.h, start, px, float(eps_first), rounds, st)
        if rc not in (OK, WARN_CG_MAXIT):
            raise self._err(rc)
        return rc, _stats_list(st)

    def cut(self):
        """Sweep cut. Returns (in_S bool [n], value, k_star)."""
        mask = np.zeros(self.n, np.uint8)
        val = C.c_double(0)
        ks = C.c_int64(0)
        rc = lib().irls_mincut_cut(self.h, mask.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(val),
                                   C.byref(ks))
        if rc != OK:
            raise self._err(rc)
        return mask.astype(bool), val.value, ks.value

    def cut_noalloc(self):
        """irls_mincut_cut_noalloc: the sweep cut in the library's static
        scratch (no device allocation). Returns (in_S bool [n], value, k_star)."""
        mask = np.zeros(self.n, np.uint8)
        val = C.c_double(0)
        ks = C.c_int64(0)
        rc = lib().irls_mincut_cut_noalloc(self.h, mask.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(val),
                                           C.byref(ks))
        if rc != OK:
            raise self._err(rc)
        return mask.astype(bool), val.value, ks.value

    def update_capacities(self, eu, ev, cap):
        """irls_mincut_update_capacities: same structure, new capacities."""
        dev = self.opt.inputs_on_device
        pu, ku, _ = _ptr_as(eu, np.int64, dev)
        pv, kv, _ = _ptr_as(ev, np.int64, dev)
        pc, kc, _ = _ptr_as(cap, np.float64, dev)
        m = 0 if ku is None else int(ku.shape[0] if hasattr(ku, "shape") else len(ku))
        rc = lib().irls_mincut_update_capacities(self.h, m, pu, pv, pc)
        if rc != OK:
            raise self._err(rc)

    def cheeger_bracket(self):
        """irls_mincut_cheeger_bracket: (lower, upper) bounds on the minimum cut."""
        lo, hi = C.c_double(0), C.c_double(0)
        rc = lib().irls_mincut_cheeger_bracket(self.h, C.byref(lo), C.byref(hi))
        if rc != OK:
            raise self._err(rc)
        return lo.value, hi.value

    def cut_two_level(self):
        """Two-level rounding (irls_mincut_cut_two_level). Returns (in_S bool [n],
        value, info dict)."""
        mask = np.zeros(self.n, np.uint8)
        val = C.c_double(0)
        info = TwoLevelInfo()
        rc = lib().irls_mincut_cut_two_level(self.h, mask.ctypes.data_as(C.POINTER(C.c_uint8)),
                                             C.byref(val), C.byref(info))
        if rc != OK:
            raise self._err(rc)
        return mask.astype(bool), val.value, {f: getattr(info, f) for f, _ in TwoLevelInfo._fields_}

    def potentials(self):
        x = np.zeros(self.n)
        rc = lib().irls_mincut_potentials(self.h, x.ctypes.data_as(C.POINTER(C.c_double)))
        if rc != OK:
            raise self._err(rc)
        return x

    def set_potentials(self, x):
        px, keep, _ = _ptr_as(x, np.float64, self.opt.inputs_on_device)
        rc = lib().irls_mincut_set_potentials(self.h, px)
        if rc != OK:
            raise self._err(rc)

    def info(self):
        nt, nnz = C.c_int64(), C.c_int64()
        fmt, K, sol, rpw = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        rc = lib().irls_mincut_info(self.h, C.byref(nt), C.byref(nnz), C.byref(fmt), C.byref(K),
                                    C.byref(sol), C.byref(rpw))
        if rc != OK:
            raise self._err(rc)
        return dict(n_nonterminal=nt.value, nnz_offdiag=nnz.value, format=fmt.value,
                    n_diagonals=K.value, solver=sol.value, rows_per_wave=rpw.value)

    SPMV_KERNELS = {0: "k_spmv_csr", 1: "k_spmv_dia", 2: "k_spmv_dia_vec", 3: "k_spmv_dia_march",
                    4: "k_spmv_dia_march"}

    def spmv_variant(self):
        """(variant, workgroups) of the CG loop's SpMV (irls_mincut_spmv_kernel)."""
        v, g = C.c_int32(), C.c_int32()
        rc = lib().irls_mincut_spmv_kernel(self.h, C.byref(v), C.byref(g))
        if rc != OK:
            raise self._err(rc)
        return v.value, g.value

    def spmv_kernel(self):
        """(kernel name, workgroups) of the CG loop's SpMV."""
        v, g = self.spmv_variant()
        return self.SPMV_KERNELS[v], g

    def time_kernel(self, which=0, reps=50):
        ms = C.c_double(0)
        rc = lib().irls_mincut_time_kernel(self.h, which, reps, C.byref(ms))
        if rc != OK:
            raise self._err(rc)
        return ms.value

    def set_march_tile(self, threads, lines):
        """irls_mincut_set_march_tile: (0, 0) restores the default shape."""
        rc = lib().irls_mincut_set_march_tile(self.h, threads, lines)
        if rc != OK:
            raise self._err(rc)

    def march_tile(self):
        """Returns (threads, lines, planes per workgroup) of the marching SpMV (zeros if none)."""
        a, b, c = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        rc = lib().irls_mincut_march_tile(self.h, C.byref(a), C.byref(b), C.byref(c))
        if rc != OK:
            raise self._err(rc)
        return a.value, b.value, c.value

    def set_kernel_timing(self, which, every=1):
        """irls_mincut_set_kernel_timing: -1 off, 0 SpMV, 1 update, 2 residual
        replacement, 3 block-Jacobi apply; launches of iterations 0, every,
        2 * every, ... are timed."""
        rc = lib().irls_mincut_set_kernel_timing(self.h, which, every)
        if rc != OK:
            raise self._err(rc)

    def kernel_timing(self):
        """Returns dict(ms_working, n_working, ms_all, n_all) of the in-solve timing."""
        mw, ma = C.c_double(0), C.c_double(0)
        nw, na = C.c_int64(0), C.c_int64(0)
        rc = lib().irls_mincut_kernel_timing(self.h, C.byref(mw), C.byref(nw), C.byref(ma), C.byref(na))
        if rc != OK:
            raise self._err(rc)
        return dict(ms_working=mw.value, n_working=nw.value, ms_all=ma.value, n_all=na.value)

    def close(self):
        if getattr(self, "h", None):
            lib().irls_mincut_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class MinCutBatch(_RowLanes):
    """Many independent graphs solved together: irls_mincut_create_batch /
    _solve_batch / _cut_batch.  `graphs` are objects with n, eu, ev, cap, s, t
    (local node ids)."""

    def __init__(self, graphs, stream=None, **opts):
        L = lib()
        self.G = len(graphs)
        self.opt = options(**opts)
        ns = [int(g.n) for g in graphs]
        ms = [int(len(g.eu)) for g in graphs]
        self.node_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
        self.edge_off = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
        cat = lambda f, dt: (np.ascontiguousarray(np.concatenate([np.asarray(getattr(g, f)) for g in graphs]), dtype=dt)
                             if self.edge_off[-1] > 0 else np.zeros(1, dt))
        self._eu, self._ev, self._cap = cat("eu", np.int64), cat("ev", np.int64), cat("cap", np.float64)
        self._s = np.array([g.s for g in graphs], np.int64)
        self._t = np.array([g.t for g in graphs], np.int64)
        P64 = C.POINTER(C.c_int64)
        h = C.c_void_p()
        rc = L.irls_mincut_create_batch(C.byref(h), self.G, self.node_off.ctypes.data_as(P64),
                                        self.edge_off.ctypes.data_as(P64), self._eu.ctypes.data_as(P64),
                                        self._ev.ctypes.data_as(P64),
                                        self._cap.ctypes.data_as(C.POINTER(C.c_double)),
                                        self._s.ctypes.data_as(P64), self._t.ctypes.data_as(P64),
                                        C.byref(self.opt), _stream_ptr(stream))
        if rc != OK:
            raise IrlsError(rc, L.irls_mincut_last_error(None).decode())
        self.h = h

    def _err(self, rc):
        return IrlsError(rc, lib().irls_mincut_last_error(self.h).decode())

    def solve(self):
        """Returns (status, stats[g][round])."""
        T1 = self.opt.rounds + 1
        st = (RoundStats * (self.G * T1))()
        rc = lib().irls_mincut_solve_batch(self.h, st)
        if rc not in (OK, WARN_CG_MAXIT):
            raise self._err(rc)
        flat = _stats_list(st)
        return rc, [flat[g * T1:(g + 1) * T1] for g in range(self.G)]

    def cut(self):
        """Returns (list of source-side masks, array of cut values)."""
        mask = np.zeros(int(self.node_off[-1]), np.uint8)
        vals = np.zeros(self.G)
        rc = lib().irls_mincut_cut_batch(self.h, mask.ctypes.data_as(C.POINTER(C.c_uint8)),
                                         vals.ctypes.data_as(C.POINTER(C.c_double)))
        if rc != OK:
            raise self._err(rc)
        m = mask.astype(bool)
        return [m[self.node_off[g]:self.node_off[g + 1]] for g in range(self.G)], vals

    def potentials(self):
        x = np.zeros(int(self.node_off[-1]))
        rc = lib().irls_mincut_potentials(self.h, x.ctypes.data_as(C.POINTER(C.c_double)))
        if rc != OK:
            raise self._err(rc)
        return [x[self.node_off[g]:self.node_off[g + 1]] for g in range(self.G)]

    def close(self):
        if getattr(self, "h", None):
            lib().irls_mincut_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Gnn:
    """Learned warm start (include/irls_gnn.h): a message-passing network that
    predicts starting potentials and a starting eps for a graph handle."""

    def __init__(self, layers=3, seed=0, stream=None, hidden=64):
        L = lib()
        h = C.c_void_p()
        rc = L.irls_gnn_create(C.byref(h), hidden, layers, C.c_uint64(seed), _stream_ptr(stream))
        if rc != OK:
            raise IrlsError(rc, L.irls_gnn_last_error(None).decode())
        self.h = h
        n = C.c_int64()
        L.irls_gnn_num_params(self.h, C.byref(n))
        self.nparams = n.value

    def _err(self, rc):
        return IrlsError(rc, lib().irls_gnn_last_error(self.h).decode())

    def get_params(self):
        p = np.zeros(self.nparams, np.float32)
        rc = lib().irls_gnn_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)))
        if rc != OK:
            raise self._err(rc)
        return p

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.shape[0] == self.nparams
        rc = lib().irls_gnn_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)))
        if rc != OK:
            raise self._err(rc)

    @staticmethod
    def _dptr(a):
        if a is None:
            return None, None
        if _is_torch(a):                      # the network's inputs are host arrays
            a = a.detach().cpu().numpy()
        a = np.ascontiguousarray(a, np.float64)
        return a.ctypes.data_as(C.POINTER(C.c_double)), a

    def predict(self, mc, intensity=None, x_start=None):
        """Returns (xhat [n] with x_s = 1, x_t = 0, log eps).  x_start None:
        the potentials mc holds."""
        x = np.zeros(mc.n)
        le = C.c_double()
        pi, ki = self._dptr(intensity)
        px, kx = self._dptr(x_start)
        rc = lib().irls_gnn_predict(self.h, mc.h, pi, px, x.ctypes.data_as(C.POINTER(C.c_double)), C.byref(le))
        if rc != OK:
            raise self._err(rc)
        return x, le.value

    def warm_start(self, mc, gamma, intensity=None):
        """Blend the prediction into the potentials mc holds (on the device);
        returns the predicted log eps."""
        pi, ki = self._dptr(intensity)
        le = C.c_double()
        rc = lib().irls_gnn_warm_start(self.h, mc.h, pi, float(gamma), C.byref(le))
        if rc != OK:
            raise self._err(rc)
        return le.value

    def loss_grad(self, mc, y, log_eps_target, lam=0.1, intensity=None, x_start=None, want_grad=False):
        _, y = self._dptr(y)
        pi, ki = self._dptr(intensity)
        px, kx = self._dptr(x_start)
        loss = C.c_double()
        g = np.zeros(self.nparams, np.float32) if want_grad else None
        rc = lib().irls_gnn_loss_grad(self.h, mc.h, pi, px, y.ctypes.data_as(C.POINTER(C.c_double)),
                                      float(log_eps_target), float(lam), C.byref(loss),
                                      None if g is None else g.ctypes.data_as(C.POINTER(C.c_float)))
        if rc != OK:
            raise self._err(rc)
        return loss.value, g

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        rc = lib().irls_gnn_adam_step(self.h, lr, beta1, beta2, eps)
        if rc != OK:
            raise self._err(rc)

    def close(self):
        if getattr(self, "h", None):
            lib().irls_gnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create_error(n, eu, ev, cap, s, t, **opts):
    """Status code irls_mincut_create returns for these arguments (0 = success)."""
    try:
        MinCut(n, eu, ev, cap, s, t, **opts).close()
        return OK
    except IrlsError as e:
        return e.code


def stream_probe(rows, reads, writes, workgroups=256, reps=20, stream=None):
    """irls_stream_probe: mean launch time (ms) of a kernel streaming `reads`
    input and `writes` output arrays of `rows` doubles."""
    ms = C.c_double(0)
    rc = lib().irls_stream_probe(int(rows), reads, writes, workgroups, reps, _stream_ptr(stream), C.byref(ms))
    if rc != OK:
        raise IrlsError(rc, lib().irls_mincut_last_error(None).decode())
    return ms.value
