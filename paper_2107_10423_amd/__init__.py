"""Python binding of libgw (include/gw.h): argument marshalling only.

Every computation happens inside libgw.so on the GPU.  The library must have
been built (``python -m paper_2107_10423_amd.build`` or
``__graft_entry__.build()``); importing this module without it raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GW_LIB_VARIANT=hostsan loads the host-sanitizer build (launch audit only)
LIB_PATH = os.path.join(_HERE, "libgw_hostsan.so" if os.environ.get("GW_LIB_VARIANT") == "hostsan"
                        else "libgw.so")

GW_PI_FP64, GW_PI_FP32, GW_PI_BF16X3 = 0, 1, 2
PREC = {"fp64": GW_PI_FP64, "fp32": GW_PI_FP32, "bf16x3": GW_PI_BF16X3}


def _prec(p):
    return PREC[p] if isinstance(p, str) else int(p)
ST_MAXITER, ST_SMALL_Z, ST_FALLBACK = 1, 2, 4

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2107_10423_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


class _Opts(ctypes.Structure):
    _fields_ = [("pi_prec", ctypes.c_int), ("minres_max_iter", ctypes.c_int),
                ("minres_rtol", ctypes.c_double), ("qp_tol", ctypes.c_double),
                ("qp_max_iter", ctypes.c_int), ("dsig_x", _dp), ("stream", ctypes.c_void_p),
                ("mem_budget_bytes", ctypes.c_size_t), ("work_budget_bytes", ctypes.c_size_t),
                ("minres_batch", ctypes.c_int), ("no_graphs", ctypes.c_int),
                ("no_precond", ctypes.c_int), ("cluster_width", ctypes.c_double),
                ("wc_prec", ctypes.c_int)]


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("xi", _dp), ("w", _dp)]


class Timing(ctypes.Structure):
    _fields_ = [("pi_ms", ctypes.c_double), ("chol_ms", ctypes.c_double),
                ("wtab_ms", ctypes.c_double), ("quad_ms", ctypes.c_double),
                ("minres_ms", ctypes.c_double), ("fallback_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("qp_rounds", ctypes.c_int),
                ("minres_iters", ctypes.c_int), ("minres_systems", ctypes.c_int),
                ("fallback_systems", ctypes.c_int), ("wtab_cached", ctypes.c_int),
                ("sd_ms", ctypes.c_double), ("sd_sweeps", ctypes.c_int),
                ("pi_kernel_ms", ctypes.c_double), ("wc_kernel_ms", ctypes.c_double),
                ("pi_launches", ctypes.c_int), ("wc_launches", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _ServerOpts(ctypes.Structure):
    _fields_ = [("pi_prec", ctypes.c_int), ("minres_max_iter", ctypes.c_int),
                ("qp_max_iter", ctypes.c_int), ("minres_rtol", ctypes.c_double),
                ("qp_tol", ctypes.c_double), ("grid_n", ctypes.c_int), ("grid_xi", _dp),
                ("grid_w", _dp), ("mem_budget_bytes", ctypes.c_size_t),
                ("n_streams", ctypes.c_int), ("work_budget_bytes", ctypes.c_size_t),
                ("wc_prec", ctypes.c_int), ("batch_max_aux", ctypes.c_int)]


class _Request(ctypes.Structure):
    _fields_ = [("n_mo", ctypes.c_int), ("n_occ", ctypes.c_int), ("n_aux", ctypes.c_int),
                ("eps", _dp), ("B_ov", _dp), ("n_rows", ctypes.c_int), ("row_ids", _ip),
                ("B_rows", _dp), ("n_states", ctypes.c_int), ("states", _ip), ("dsig_x", _dp)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("rc", ctypes.c_int), ("footprint_bytes", ctypes.c_size_t),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("slot", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_ulonglong), ("completed", ctypes.c_ulonglong),
                ("failed", ctypes.c_ulonglong), ("budget_bytes", ctypes.c_size_t),
                ("reserved_bytes", ctypes.c_size_t), ("peak_reserved_bytes", ctypes.c_size_t),
                ("active", ctypes.c_int), ("peak_active", ctypes.c_int),
                ("batches", ctypes.c_long), ("batched_requests", ctypes.c_long),
                ("graph_replays", ctypes.c_long), ("device_mallocs", ctypes.c_long),
                ("cache_hits", ctypes.c_long), ("device_frees", ctypes.c_long),
                ("cached_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_ctxp = ctypes.c_void_p
_sig = {
    "gw_last_error": (ctypes.c_char_p, []),
    "gw_grid_gauss_legendre": (ctypes.c_int, [ctypes.c_int, ctypes.c_double, _dp, _dp]),
    "gw_setup": (ctypes.c_int, [ctypes.POINTER(_ctxp), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                _dp, _dp, ctypes.c_int, _ip, _dp, ctypes.POINTER(_Opts)]),
    "gw_setup_full": (ctypes.c_int, [ctypes.POINTER(_ctxp), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _dp, _dp, ctypes.POINTER(_Opts)]),
    "gw_setup_uhf": (ctypes.c_int, [ctypes.POINTER(_ctxp), ctypes.c_int, _ip, ctypes.c_int, _dp,
                                    _dp, _dp, ctypes.c_int, _ip, _dp, ctypes.POINTER(_Opts)]),
    "gw_qp": (ctypes.c_int, [_ctxp, ctypes.c_int, _ip, ctypes.POINTER(_Grid), _dp, _dp, _dp, _ip]),
    "gw_evgw": (ctypes.c_int, [_ctxp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                               _ip, ctypes.POINTER(_Grid), _dp, _dp, _dp, _ip, _dp, _ip]),
    "gw_qp_sd": (ctypes.c_int, [_ctxp, ctypes.c_int, _ip, _dp, _dp, _dp, _ip]),
    "gw_rpa_excitations": (ctypes.c_int, [_ctxp, _dp]),
    "gw_free": (None, [_ctxp]),
    "gw_set_pi_prec": (ctypes.c_int, [_ctxp, ctypes.c_int]),
    "gw_dielectric": (ctypes.c_int, [_ctxp, ctypes.c_int, _dp, _dp]),
    "gw_dielectric_noalloc": (ctypes.c_int, [_ctxp, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_long, ctypes.c_long]),
    "gw_cholesky": (ctypes.c_int, [_ctxp, ctypes.c_int, _dp, _dp]),
    "gw_wtable": (ctypes.c_int, [_ctxp, ctypes.POINTER(_Grid), _dp]),
    "gw_sigma": (ctypes.c_int, [_ctxp, ctypes.c_int, _ip, _dp, ctypes.POINTER(_Grid), _dp, _dp, _ip]),
    "gw_residues": (ctypes.c_int, [_ctxp, ctypes.c_int, _ip, _ip, _dp, ctypes.c_int, _dp, _dp,
                                   _dp, _ip]),
    "gw_get_timing": (ctypes.c_int, [_ctxp, ctypes.POINTER(Timing)]),
    "gw_reset_cache": (ctypes.c_int, [_ctxp]),
    "gw_footprint": (ctypes.c_size_t, [ctypes.c_int] * 6 + [ctypes.POINTER(_Opts)]),
    "gw_server_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(_ServerOpts)]),
    "gw_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(_Request),
                                        ctypes.POINTER(ctypes.c_ulonglong)]),
    "gw_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_ulonglong, _dp, _dp, _dp, _ip,
                                      ctypes.POINTER(RequestInfo)]),
    "gw_server_drain": (ctypes.c_int, [ctypes.c_void_p]),
    "gw_server_get_stats": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ServerStats)]),
    "gw_server_clock": (ctypes.c_double, [ctypes.c_void_p]),
    "gw_server_destroy": (None, [ctypes.c_void_p]),
    "gw_audit_enable": (ctypes.c_int, []),
    "gw_audit_launch_count": (ctypes.c_long, []),
    "gw_group_stage_a": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_ctxp), ctypes.POINTER(_Grid),
                                        ctypes.c_int, _ip]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class GWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libgw error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise GWError(rc, _lib.gw_last_error().decode())


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _pd(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _pi(a):
    return a.ctypes.data_as(_ip) if a is not None else None


def grid_gauss_legendre(n: int, x0: float = 0.5):
    xi = np.empty(n)
    w = np.empty(n)
    _check(_lib.gw_grid_gauss_legendre(int(n), float(x0), _pd(xi), _pd(w)))
    return xi, w


class Grid:
    def __init__(self, xi, w):
        self.xi = _d(xi)
        self.w = _d(w)
        if self.xi.shape != self.w.shape or self.xi.ndim != 1:
            raise ValueError("grid arrays must be 1-D and of equal length")
        self._g = _Grid(len(self.xi), _pd(self.xi), _pd(self.w))

    @classmethod
    def gauss_legendre(cls, n, x0=0.5):
        return cls(*grid_gauss_legendre(n, x0))

    @property
    def n(self):
        return len(self.xi)


class Context:
    """One molecule resident on the GPU (wraps gw_setup / gw_free)."""

    def __init__(self, eps, n_occ, B_ov, row_ids, B_rows, pi_prec="fp64", minres_max_iter=0,
                 minres_rtol=0.0, qp_tol=0.0, qp_max_iter=0, dsig_x=None, stream=None,
                 mem_budget_bytes=0, work_budget_bytes=0, minres_batch=0, graphs=True,
                 cluster_width=0.0, precond=True, wc_prec="fp64"):
        eps = _d(eps)
        B_ov = _d(B_ov)
        rows = _i(row_ids)
        B_rows = _d(B_rows)
        n_mo = eps.size
        n_aux = B_ov.shape[0]
        if B_ov.shape != (n_aux, n_occ * (n_mo - n_occ)):
            raise ValueError("B_ov must be [n_aux][n_occ*n_virt]")
        if B_rows.shape != (rows.size, n_mo, n_aux):
            raise ValueError("B_rows must be [n_rows][n_mo][n_aux]")
        o = self._make_opts(pi_prec, minres_max_iter, minres_rtol, qp_tol, qp_max_iter,
                            dsig_x, stream, mem_budget_bytes, work_budget_bytes, minres_batch,
                            graphs, cluster_width, precond, wc_prec)
        h = _ctxp()
        _check(_lib.gw_setup(ctypes.byref(h), n_mo, int(n_occ), n_aux, _pd(eps), _pd(B_ov),
                             rows.size, _pi(rows), _pd(B_rows), ctypes.byref(o)))
        self._h = h
        self.n_mo, self.n_occ, self.n_aux = n_mo, int(n_occ), n_aux
        self.row_ids = rows.copy()

    def _make_opts(self, pi_prec="fp64", minres_max_iter=0, minres_rtol=0.0, qp_tol=0.0,
                   qp_max_iter=0, dsig_x=None, stream=None, mem_budget_bytes=0,
                   work_budget_bytes=0, minres_batch=0, graphs=True, cluster_width=0.0,
                   precond=True, wc_prec="fp64"):
        self._dsx = _d(dsig_x) if dsig_x is not None else None
        return _Opts(_prec(pi_prec),
                     int(minres_max_iter), float(minres_rtol), float(qp_tol), int(qp_max_iter),
                     _pd(self._dsx), ctypes.c_void_p(stream) if stream else None,
                     int(mem_budget_bytes), int(work_budget_bytes), int(minres_batch),
                     0 if graphs else 1, 0 if precond else 1, float(cluster_width),
                     _prec(wc_prec))

    @classmethod
    def from_inputs(cls, inp, **kw):
        return cls(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, **kw)

    @classmethod
    def full(cls, eps, n_occ, B, **kw):
        """Context from the full symmetric B [n_aux][n_mo][n_mo] (gw_setup_full):
        every state may be requested."""
        self = cls.__new__(cls)
        self._h = None
        eps = _d(eps)
        B = _d(B)
        n_mo = eps.size
        if B.ndim != 3 or B.shape[1:] != (n_mo, n_mo):
            raise ValueError("B must be [n_aux][n_mo][n_mo]")
        o = self._make_opts(**kw)
        h = _ctxp()
        _check(_lib.gw_setup_full(ctypes.byref(h), n_mo, int(n_occ), B.shape[0], _pd(eps),
                                  _pd(B), ctypes.byref(o)))
        self._h = h
        self.n_mo, self.n_occ, self.n_aux = n_mo, int(n_occ), B.shape[0]
        self.row_ids = np.arange(n_mo, dtype=np.int32)
        return self

    @classmethod
    def uhf(cls, eps, n_occ, B_ov_up, B_ov_down, row_ids, B_rows, **kw):
        """Open-shell context (gw_setup_uhf): eps [2][n_mo], n_occ (up, down),
        row ids and states as spin-orbital indices sigma * n_mo + n."""
        self = cls.__new__(cls)
        self._h = None
        eps = _d(eps)
        if eps.ndim != 2 or eps.shape[0] != 2:
            raise ValueError("eps must be [2][n_mo]")
        n_mo = eps.shape[1]
        occ = _i(list(n_occ))
        Bs = [_d(B_ov_up), _d(B_ov_down)]
        n_aux = Bs[0].shape[0]
        for sp in (0, 1):
            if Bs[sp].shape != (n_aux, int(occ[sp]) * (n_mo - int(occ[sp]))):
                raise ValueError(f"B_ov of spin {sp} must be [n_aux][n_occ*n_virt]")
        rows = _i(row_ids)
        B_rows = _d(B_rows)
        if B_rows.shape != (rows.size, n_mo, n_aux):
            raise ValueError("B_rows must be [n_rows][n_mo][n_aux]")
        o = self._make_opts(**kw)
        h = _ctxp()
        _check(_lib.gw_setup_uhf(ctypes.byref(h), n_mo, _pi(occ), n_aux, _pd(eps), _pd(Bs[0]),
                                 _pd(Bs[1]), rows.size, _pi(rows), _pd(B_rows),
                                 ctypes.byref(o)))
        self._h = h
        self.n_mo, self.n_occ, self.n_aux = n_mo, (int(occ[0]), int(occ[1])), n_aux
        self.row_ids = rows.copy()
        return self

    @classmethod
    def from_inputs_uhf(cls, inp, **kw):
        return cls.uhf(inp.eps, inp.n_occ, inp.B_ov[0], inp.B_ov[1], inp.row_ids, inp.B_rows,
                       **kw)

    def close(self):
        if getattr(self, "_h", None):
            _lib.gw_free(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_pi_prec(self, prec):
        _check(_lib.gw_set_pi_prec(self._h, PREC[prec] if isinstance(prec, str) else int(prec)))

    def qp(self, states: Sequence[int], grid: Grid):
        st = _i(states)
        n = st.size
        E, S, Z = np.empty(n), np.empty(n), np.empty(n)
        status = np.empty(n, dtype=np.int32)
        _check(_lib.gw_qp(self._h, n, _pi(st), ctypes.byref(grid._g), _pd(E), _pd(S), _pd(Z),
                          _pi(status)))
        return E, S, Z, status

    def evgw(self, states: Sequence[int], grid: Grid, mode="evgw0", n_cycles=3, ev_tol=0.0):
        """Eigenvalue self-consistent GW (gw_evgw).  Returns (E, sigma_c, Z, status)
        of the last cycle and the QP energies of every cycle, [cycles][n_states]."""
        st = _i(states)
        n = st.size
        m = {"evgw0": 0, "evgw": 1}[mode] if isinstance(mode, str) else int(mode)
        E, S, Z = np.empty(n), np.empty(n), np.empty(n)
        status = np.empty(n, dtype=np.int32)
        hist = np.zeros((max(int(n_cycles), 1), n))
        done = ctypes.c_int(0)
        _check(_lib.gw_evgw(self._h, m, int(n_cycles), float(ev_tol), n, _pi(st),
                            ctypes.byref(grid._g), _pd(E), _pd(S), _pd(Z), _pi(status), _pd(hist),
                            ctypes.byref(done)))
        return E, S, Z, status, hist[:done.value].copy()

    def qp_sd(self, states: Sequence[int]):
        """G0W0 by the spectral-decomposition route (gw_qp_sd)."""
        st = _i(states)
        n = st.size
        E, S, Z = np.empty(n), np.empty(n), np.empty(n)
        status = np.empty(n, dtype=np.int32)
        _check(_lib.gw_qp_sd(self._h, n, _pi(st), _pd(E), _pd(S), _pd(Z), _pi(status)))
        return E, S, Z, status

    def rpa_excitations(self):
        """Casida excitation energies Omega_s, ascending (gw_rpa_excitations)."""
        occ = self.n_occ if isinstance(self.n_occ, tuple) else (self.n_occ,)
        n_ov = sum(o * (self.n_mo - o) for o in occ)
        out = np.empty(n_ov)
        _check(_lib.gw_rpa_excitations(self._h, _pd(out)))
        return out

    def wtable(self, grid: Grid):
        out = np.empty((self.row_ids.size, self.n_mo, grid.n))
        _check(_lib.gw_wtable(self._h, ctypes.byref(grid._g), _pd(out)))
        return out

    def dielectric(self, xi):
        xi = _d(np.atleast_1d(xi))
        out = np.empty((xi.size, self.n_aux, self.n_aux))
        _check(_lib.gw_dielectric(self._h, xi.size, _pd(xi), _pd(out)))
        return out

    def dielectric_noalloc(self, d_xi, n_xi, d_out, ld_out, out_stride):
        """gw_dielectric_noalloc: device pointers (ints) in and out, nothing
        allocated; asynchronous on the context's stream."""
        _check(_lib.gw_dielectric_noalloc(self._h, int(n_xi), ctypes.c_void_p(d_xi),
                                          ctypes.c_void_p(d_out), int(ld_out), int(out_stride)))

    def cholesky(self, xi):
        xi = _d(np.atleast_1d(xi))
        out = np.empty((xi.size, self.n_aux, self.n_aux))
        _check(_lib.gw_cholesky(self._h, xi.size, _pd(xi), _pd(out)))
        return out

    def sigma(self, states, omega, grid: Grid):
        st = _i(states)
        om = _d(omega)
        n = st.size
        s, ds = np.empty(n), np.empty(n)
        nres = np.empty(n, dtype=np.int32)
        _check(_lib.gw_sigma(self._h, n, _pi(st), _pd(om), ctypes.byref(grid._g), _pd(s), _pd(ds),
                             _pi(nres)))
        return s, ds, nres

    def residues(self, states, m, w, use_fallback=True):
        st, mm, ww = _i(states), _i(m), _d(w)
        k = st.size
        x = np.empty((k, self.n_aux))
        wc, dwc = np.empty(k), np.empty(k)
        it = np.empty(k, dtype=np.int32)
        _check(_lib.gw_residues(self._h, k, _pi(st), _pi(mm), _pd(ww), int(bool(use_fallback)),
                                _pd(x), _pd(wc), _pd(dwc), _pi(it)))
        return x, wc, dwc, it

    def reset_cache(self):
        _check(_lib.gw_reset_cache(self._h))

    def timing(self):
        t = Timing()
        _check(_lib.gw_get_timing(self._h, ctypes.byref(t)))
        return t.as_dict()


GW_EAUDIT = -5


def footprint(n_mo, n_occ, n_aux, n_rows, n_states, grid_n, pi_prec="fp64", work_budget_bytes=0,
              minres_batch=0, wc_prec="fp64"):
    """gw_footprint: device bytes a context of these sizes uses."""
    o = _Opts(_prec(pi_prec), 0, 0.0, 0.0, 0, None, None, 0, int(work_budget_bytes),
              int(minres_batch), 0, 0, 0.0, _prec(wc_prec))
    return int(_lib.gw_footprint(n_mo, n_occ, n_aux, n_rows, n_states, grid_n, ctypes.byref(o)))


class Server:
    """Request server (gw_server_*): submit molecules, poll results."""

    def __init__(self, grid, pi_prec="fp64", mem_budget_bytes=0, n_streams=0,
                 work_budget_bytes=0, qp_tol=0.0, minres_rtol=0.0, wc_prec="fp64",
                 batch_max_aux=0):
        self._grid = grid
        o = _ServerOpts(_prec(pi_prec), 0, 0,
                        float(minres_rtol), float(qp_tol), grid.n, _pd(grid.xi), _pd(grid.w),
                        int(mem_budget_bytes), int(n_streams), int(work_budget_bytes),
                        _prec(wc_prec), int(batch_max_aux))
        h = ctypes.c_void_p()
        _check(_lib.gw_server_create(ctypes.byref(h), ctypes.byref(o)))
        self._h = h
        self._n = {}

    def submit(self, eps, n_occ, B_ov, row_ids, B_rows, states, dsig_x=None):
        eps, B_ov, rows, B_rows, st = _d(eps), _d(B_ov), _i(row_ids), _d(B_rows), _i(states)
        dsx = _d(dsig_x) if dsig_x is not None else None
        q = _Request(eps.size, int(n_occ), B_ov.shape[0], _pd(eps), _pd(B_ov), rows.size,
                     _pi(rows), _pd(B_rows), st.size, _pi(st), _pd(dsx))
        t = ctypes.c_ulonglong()
        _check(_lib.gw_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        self._n[t.value] = st.size
        return t.value

    def submit_inputs(self, inp, states):
        return self.submit(inp.eps, inp.n_occ, inp.B_ov, inp.row_ids, inp.B_rows, states)

    def poll(self, ticket):
        """None while pending, else (E, sigma_c, Z, status, info dict)."""
        n = self._n[ticket]
        E, S, Z = np.empty(n), np.empty(n), np.empty(n)
        st = np.empty(n, dtype=np.int32)
        info = RequestInfo()
        rc = _lib.gw_server_poll(self._h, ticket, _pd(E), _pd(S), _pd(Z), _pi(st),
                                 ctypes.byref(info))
        if rc == 1:
            return None
        _check(rc)
        del self._n[ticket]
        return E, S, Z, st, info.as_dict()

    def drain(self):
        _check(_lib.gw_server_drain(self._h))

    def stats(self):
        s = ServerStats()
        _check(_lib.gw_server_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def clock(self):
        return float(_lib.gw_server_clock(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.gw_server_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def audit_enable():
    """Irreversibly switch this process into launch-audit mode (include/gw_audit.h)."""
    _check(_lib.gw_audit_enable())


def audit_launch_count():
    return int(_lib.gw_audit_launch_count())


def group_stage_a(contexts, grid, use_graph=True):
    """The server's grouped stage A on contexts of one padded shape
    (gw_group_stage_a): one batched launch sequence over all their grid points;
    returns each context's status (0: its W^c table is cached)."""
    n = len(contexts)
    arr = (_ctxp * n)(*[c._h for c in contexts])
    rc = np.zeros(n, dtype=np.int32)
    _check(_lib.gw_group_stage_a(n, arr, ctypes.byref(grid._g), int(bool(use_graph)), _pi(rc)))
    return rc


def exported_symbols():
    """Names declared in include/gw.h that the loaded library exports."""
    return sorted(n for n in _sig if hasattr(_lib, n))
