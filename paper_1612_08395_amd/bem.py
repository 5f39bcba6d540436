"""ctypes binding of libbem.so (the C ABI declared in include/bem.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Importing this module fails loudly if the library has not been
built (``python -m paper_1612_08395_amd.build``); there is no fallback.

Function names follow the C ABI.  Host arrays are numpy float64 arrays of
shape (ny, nx); device arrays are anything with ``data_ptr()`` (torch
tensors on the GPU) or a raw integer address.
"""
import ctypes
import os

import numpy as np

# torch ships its own HIP runtime (SONAME libamdhip64.so.7) and loads it under
# the unversioned file name.  Importing torch first makes the dynamic linker
# bind libbem.so's libamdhip64.so.7 dependency to that same runtime, so device
# pointers and streams handed over from torch belong to the runtime that
# launches the library's kernels (two runtimes in one process cannot share
# the device).
import torch  # noqa: F401  (must precede the CDLL below)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbem.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1612_08395_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

BEM_OK, BEM_ENOCONV, BEM_EFLOOR = 0, 1, 2
BEM_EINVAL, BEM_ENOMEM, BEM_EDEVICE, BEM_EUNSUPPORTED, BEM_ENUMERIC = -1, -2, -3, -4, -5
BEM_FP64, BEM_MIXED = 0, 1
BEM_MAX_N = 4096

_c_int, _c_double, _vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bem error {code}: {msg}")
        self.code = code


class InfluenceInfo(ctypes.Structure):
    _fields_ = [("nx", _c_int), ("ny", _c_int), ("Mx", _c_int), ("My", _c_int),
                ("dx", _c_double), ("dy", _c_double), ("k", _c_double), ("nu", _c_double),
                ("E0", _c_double), ("c0", _c_double),
                ("alpha", _c_double), ("C", _c_double), ("K00", _c_double),
                ("device_bytes", ctypes.c_longlong)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_lib_last_error = _sig("bem_last_error", ctypes.c_char_p, [])
_f_influence_ex = _sig("bem_influence_ex", _c_int,
                       [_c_int, _c_int, _c_double, _c_double, _c_double, _c_double, _c_double,
                        _c_double, ctypes.POINTER(_vp)])
_f_influence = _sig("bem_influence", _c_int,
                    [_c_int, _c_int, _c_double, _c_double, _c_double, ctypes.POINTER(_vp)])
_f_influence_free = _sig("bem_influence_free", _c_int, [_vp])
_f_influence_info = _sig("bem_influence_info", _c_int, [_vp, ctypes.POINTER(InfluenceInfo)])
_f_influence_coeffs = _sig("bem_influence_coeffs", _c_int, [_vp, _dp])
_f_convolve = _sig("bem_convolve", _c_int, [_vp, _dp, _dp, _vp])
_f_convolve_dev = _sig("bem_convolve_dev", _c_int, [_vp, _c_int, _vp, _vp, _vp])
_f_convolve_dev_noalloc = _sig("bem_convolve_dev_noalloc", _c_int, [_vp, _c_int, _vp, _vp, _vp])
BEM_NOALLOC_SCRATCH_BYTES = 16 << 20


def bem_last_error():
    return _lib_last_error().decode()


def _check(rc, warn_ok=True):
    if rc < 0 or (rc > 0 and not warn_ok):
        raise BemError(rc, bem_last_error())
    return rc


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _host(a, shape):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


class Influence:
    """Owning wrapper of a bem_influence_t handle."""

    def __init__(self, handle):
        self._h = handle
        info = InfluenceInfo()
        _check(_f_influence_info(self._h, ctypes.byref(info)))
        self.info = info
        self.nx, self.ny = info.nx, info.ny

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            _f_influence_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def bem_influence_ex(nx, ny, dx, dy, k, nu, E0=1.0, c0=1.0):
    h = _vp()
    _check(_f_influence_ex(int(nx), int(ny), float(dx), float(dy), float(k), float(nu),
                           float(E0), float(c0), ctypes.byref(h)))
    return Influence(h)


def bem_influence(nx, ny, dx, k, nu):
    h = _vp()
    _check(_f_influence(int(nx), int(ny), float(dx), float(k), float(nu), ctypes.byref(h)))
    return Influence(h)


def bem_influence_free(K):
    K.free()


def bem_influence_info(K):
    return K.info


def bem_influence_coeffs(K):
    out = np.empty((2 * K.ny - 1, 2 * K.nx - 1))
    _check(_f_influence_coeffs(K.handle, out.ctypes.data_as(_dp)))
    return out


def bem_convolve(K, p, stream=None):
    p = _host(p, (K.ny, K.nx))
    u = np.empty_like(p)
    _check(_f_convolve(K.handle, p.ctypes.data_as(_dp), u.ctypes.data_as(_dp), _stream(stream)))
    return u


def bem_convolve_dev(K, precision, p, u, stream=None):
    _check(_f_convolve_dev(K.handle, int(precision), _ptr(p), _ptr(u), _stream(stream)))


def bem_convolve_dev_noalloc(K, precision, p, u, stream=None):
    _check(_f_convolve_dev_noalloc(K.handle, int(precision), _ptr(p), _ptr(u), _stream(stream)))


# ---- contact solves ----------------------------------------------------------

BEM_CTRL_INDENT, BEM_CTRL_FORCE = 0, 1


class Params(ctypes.Structure):
    _fields_ = [("control", _c_int), ("precision", _c_int),
                ("d", _c_double), ("F", _c_double), ("gamma", _c_double),
                ("p_crit", _c_double), ("d_preload", _c_double), ("tol", _c_double),
                ("max_iter", _c_int), ("stall_limit", _c_int)]


class Result(ctypes.Structure):
    _fields_ = [("F", _c_double), ("area", _c_double), ("d", _c_double),
                ("residual", _c_double), ("p_crit", _c_double),
                ("n_contact", ctypes.c_longlong), ("n_penetrating", ctypes.c_longlong),
                ("iters", _c_int), ("detach_rounds", _c_int), ("status", _c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_u8p = ctypes.POINTER(ctypes.c_ubyte)
_f_params_init = _sig("bem_params_init", None, [ctypes.POINTER(Params)])
_f_state_create = _sig("bem_state_create", _c_int, [_vp, ctypes.POINTER(_vp)])
_f_state_free = _sig("bem_state_free", _c_int, [_vp])
_f_state_set = _sig("bem_state_set", _c_int, [_vp, _dp, _u8p])
_f_state_get = _sig("bem_state_get", _c_int, [_vp, _dp, _u8p])
_f_solve = _sig("bem_solve", _c_int, [_vp, _dp, ctypes.POINTER(Params), _vp, _dp, _u8p, _dp,
                                      ctypes.POINTER(Result), _vp])
_f_solve_dev = _sig("bem_solve_dev", _c_int, [_vp, _vp, ctypes.POINTER(Params), _vp, _vp, _vp,
                                              _vp, ctypes.POINTER(Result), _vp])
_f_sweep = _sig("bem_sweep", _c_int, [_vp, _dp, ctypes.POINTER(Params), _dp, _c_int, _vp,
                                      ctypes.POINTER(Result), _vp])
_f_sweep_dev = _sig("bem_sweep_dev", _c_int, [_vp, _vp, ctypes.POINTER(Params), _dp, _c_int,
                                              _c_int, _vp, ctypes.POINTER(Result), _vp])
_f_c1 = _sig("bem_c1", _c_double, [_c_double])
_f_p_crit = _sig("bem_p_crit", _c_double, [_c_double, _c_double, _c_double, _c_double,
                                           _c_double, _c_double])


def bem_params_init(**kw):
    """Default parameters, overridden by keyword (d=..., precision=..., gamma=...)."""
    prm = Params()
    _f_params_init(ctypes.byref(prm))
    for key, val in kw.items():
        if not hasattr(prm, key):
            raise AttributeError(key)
        setattr(prm, key, val)
    return prm


class State:
    """Owning wrapper of a bem_state_t handle (warm-start pressure and contact set)."""

    def __init__(self, K):
        self.K = K
        h = _vp()
        _check(_f_state_create(K.handle, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def free(self):
        if self._h:
            _f_state_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def bem_state_create(K):
    return State(K)


def bem_state_free(st):
    st.free()


def bem_state_set(st, p=None, contact=None):
    shape = (st.K.ny, st.K.nx)
    pp = _host(p, shape).ctypes.data_as(_dp) if p is not None else None
    cc = None
    if contact is not None:
        c = np.ascontiguousarray(contact, dtype=np.uint8)
        if c.shape != shape:
            raise ValueError("contact shape")
        cc = c.ctypes.data_as(_u8p)
    _check(_f_state_set(st.handle, pp, cc))


def bem_state_get(st):
    shape = (st.K.ny, st.K.nx)
    p = np.empty(shape)
    c = np.empty(shape, dtype=np.uint8)
    _check(_f_state_get(st.handle, p.ctypes.data_as(_dp), c.ctypes.data_as(_u8p)))
    return p, c


def bem_solve(K, h, prm, state=None, want_u=False, stream=None):
    """Returns (status, result, p, contact, u or None) with host arrays."""
    shape = (K.ny, K.nx)
    h = _host(h, shape)
    p = np.empty(shape)
    c = np.empty(shape, dtype=np.uint8)
    u = np.empty(shape) if want_u else None
    res = Result()
    rc = _f_solve(K.handle, h.ctypes.data_as(_dp), ctypes.byref(prm),
                  state.handle if state is not None else None,
                  p.ctypes.data_as(_dp), c.ctypes.data_as(_u8p),
                  u.ctypes.data_as(_dp) if u is not None else None, ctypes.byref(res),
                  _stream(stream))
    _check(rc)
    return rc, res, p, c, u


def bem_solve_dev(K, h, prm, state=None, p_out=None, contact_out=None, u_out=None, stream=None):
    """Device arrays (torch tensors or addresses): h, p_out, u_out float64;
    contact_out uint8.  Returns (status, result)."""
    res = Result()
    rc = _f_solve_dev(K.handle, _ptr(h), ctypes.byref(prm),
                      state.handle if state is not None else None,
                      _ptr(p_out), _ptr(contact_out), _ptr(u_out), ctypes.byref(res),
                      _stream(stream))
    _check(rc)
    return rc, res


def bem_sweep(K, h, prm, d_list, state=None, stream=None):
    """Returns (status, [Result, ...])."""
    h = _host(h, (K.ny, K.nx))
    d = np.ascontiguousarray(d_list, dtype=np.float64)
    res = (Result * len(d))()
    rc = _f_sweep(K.handle, h.ctypes.data_as(_dp), ctypes.byref(prm), d.ctypes.data_as(_dp),
                  len(d), state.handle if state is not None else None, res, _stream(stream))
    _check(rc)
    return rc, list(res)


def bem_sweep_dev(K, h, prm, d_list, chains=1, state=None, stream=None):
    """h: device array (float64, ny x nx).  Returns (status, [Result, ...])."""
    d = np.ascontiguousarray(d_list, dtype=np.float64)
    res = (Result * len(d))()
    rc = _f_sweep_dev(K.handle, _ptr(h), ctypes.byref(prm), d.ctypes.data_as(_dp), len(d),
                      int(chains), state.handle if state is not None else None, res,
                      _stream(stream))
    _check(rc)
    return rc, list(res)


def bem_c1(k):
    return _f_c1(float(k))


def bem_p_crit(k, nu, gamma, dx, E0=1.0, c0=1.0):
    return _f_p_crit(float(k), float(nu), float(gamma), float(dx), float(E0), float(c0))


_f_kernel_time = _sig("bem_kernel_time", _c_int, [_vp, _c_int, _c_int, _c_int, _vp,
                                                  ctypes.POINTER(_c_double)])


def bem_kernel_time(K, precision, which, reps=20, stream=None):
    """Average ms of one convolution sweep kernel (0 R2C, 1 column, 2 C2R,
    3 column spectral energy)."""
    ms = _c_double()
    _check(_f_kernel_time(K.handle, int(precision), int(which), int(reps), _stream(stream),
                          ctypes.byref(ms)))
    return ms.value


class Clock(ctypes.Structure):
    """Per-launch-kind totals of the solver clock; kinds in CG-iteration order:
    update+R2C, column, C2R+gap, direction+R2C, column, C2R+dots."""
    _fields_ = [("iterations", ctypes.c_longlong), ("launches", ctypes.c_longlong * 6),
                ("ms", _c_double * 6), ("skipped", ctypes.c_longlong),
                ("skipped_ms", _c_double), ("shifts", ctypes.c_longlong),
                ("shift_ms", _c_double)]

    KINDS = ("update_r2c", "column", "gap_c2r", "direction_r2c", "column", "dots_c2r")

    def as_dict(self):
        return {"iterations": self.iterations, "launches": list(self.launches),
                "ms": list(self.ms), "skipped": self.skipped, "skipped_ms": self.skipped_ms,
                "shifts": self.shifts, "shift_ms": self.shift_ms}

    def loop_ms(self):
        """Device time of the iterations worked on, gap shifts included."""
        return sum(self.ms) + self.shift_ms


_f_clock_start = _sig("bem_clock_start", _c_int, [])
_f_clock_stop = _sig("bem_clock_stop", _c_int, [ctypes.POINTER(Clock)])


def bem_clock_start():
    _check(_f_clock_start())


def bem_clock_stop():
    c = Clock()
    _check(_f_clock_stop(ctypes.byref(c)))
    return c


# ---- serving -----------------------------------------------------------------

class Request(ctypes.Structure):
    _fields_ = [("nx", _c_int), ("ny", _c_int), ("dx", _c_double), ("dy", _c_double),
                ("k", _c_double), ("nu", _c_double), ("E0", _c_double), ("c0", _c_double),
                ("h", _dp), ("prm", Params), ("p_out", _dp), ("contact_out", _u8p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("queued", ctypes.c_longlong), ("running", _c_int), ("peak_running", _c_int),
                ("p50_latency_s", _c_double), ("p99_latency_s", _c_double),
                ("mean_wait_s", _c_double), ("solves_per_s", _c_double),
                ("device_bytes_reserved", ctypes.c_longlong),
                ("cache_entries", ctypes.c_longlong), ("cache_hits", ctypes.c_longlong),
                ("cache_misses", ctypes.c_longlong), ("evictions", ctypes.c_longlong),
                ("batched", ctypes.c_longlong), ("mean_batch_slots", _c_double),
                ("engine_launch_s", _c_double), ("engine_sync_s", _c_double),
                ("engine_step_s", _c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_llp = ctypes.POINTER(ctypes.c_longlong)
_f_state_reset = _sig("bem_state_reset", _c_int, [_vp])
_f_footprint = _sig("bem_footprint", _c_int, [_c_int, _c_int, _c_int, _llp, _llp])
_f_server_create = _sig("bem_server_create", _c_int, [ctypes.c_longlong, _c_int,
                                                      ctypes.POINTER(_vp)])
_f_server_create_ex = _sig("bem_server_create_ex", _c_int, [ctypes.c_longlong, _c_int, _c_int,
                                                            ctypes.POINTER(_vp)])
_f_server_submit = _sig("bem_server_submit", _c_int, [_vp, ctypes.POINTER(Request), _llp])
_f_server_session_open = _sig("bem_server_session_open", _c_int, [_vp, _llp])
_f_server_submit_session = _sig("bem_server_submit_session", _c_int,
                                [_vp, ctypes.c_longlong, ctypes.POINTER(Request), _llp])
_f_server_session_close = _sig("bem_server_session_close", _c_int, [_vp, ctypes.c_longlong])
_f_server_poll = _sig("bem_server_poll", _c_int, [_vp, ctypes.c_longlong, _c_int,
                                                  ctypes.POINTER(Result), ctypes.POINTER(_c_int)])
_f_server_stats = _sig("bem_server_stats", _c_int, [_vp, ctypes.POINTER(ServerStats)])
_f_server_reset_stats = _sig("bem_server_reset_stats", _c_int, [_vp])
_f_server_free = _sig("bem_server_free", _c_int, [_vp])


def bem_state_reset(st):
    _check(_f_state_reset(st.handle))


def bem_footprint(nx, ny, precision):
    a, b = ctypes.c_longlong(), ctypes.c_longlong()
    _check(_f_footprint(int(nx), int(ny), int(precision), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


class Server:
    """Owning wrapper of bem_server_t.  Keeps each submitted request's host
    arrays alive until the request has been polled."""

    def __init__(self, budget_bytes, n_slots, batch_slots=None):
        h = _vp()
        if batch_slots is None:
            _check(_f_server_create(int(budget_bytes), int(n_slots), ctypes.byref(h)))
        else:
            _check(_f_server_create_ex(int(budget_bytes), int(n_slots), int(batch_slots),
                                       ctypes.byref(h)))
        self._h = h
        self._keep = {}

    @property
    def handle(self):
        return self._h

    def submit(self, nx, ny, dx, k, nu, h, prm, dy=None, E0=1.0, c0=1.0, want_p=False,
               session=None):
        """Queue a request (bem_server_submit), or with `session` a request of
        that session (bem_server_submit_session); returns its id."""
        h = _host(h, (ny, nx))
        p = np.empty((ny, nx)) if want_p else None
        c = np.empty((ny, nx), dtype=np.uint8) if want_p else None
        req = Request(nx, ny, dx, dx if dy is None else dy, k, nu, E0, c0,
                      h.ctypes.data_as(_dp), prm,
                      p.ctypes.data_as(_dp) if p is not None else None,
                      c.ctypes.data_as(_u8p) if c is not None else None)
        rid = ctypes.c_longlong()
        if session is None:
            _check(_f_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid)))
        else:
            _check(_f_server_submit_session(self._h, int(session), ctypes.byref(req),
                                            ctypes.byref(rid)))
        self._keep[rid.value] = (p, c)
        return rid.value

    def session_open(self):
        """bem_server_session_open: a session id."""
        sid = ctypes.c_longlong()
        _check(_f_server_session_open(self._h, ctypes.byref(sid)))
        return sid.value

    def session_close(self, session):
        _check(_f_server_session_close(self._h, int(session)))

    def poll(self, rid, wait=True):
        """None while pending (wait=False), else (status, Result, p, contact)."""
        res = Result()
        st = _c_int()
        rc = _f_server_poll(self._h, int(rid), 1 if wait else 0, ctypes.byref(res), ctypes.byref(st))
        _check(rc)
        if rc == 1:
            return None
        p, c = self._keep.pop(rid)
        return st.value, res, p, c

    def stats(self):
        s = ServerStats()
        _check(_f_server_stats(self._h, ctypes.byref(s)))
        return s

    def reset_stats(self):
        _check(_f_server_reset_stats(self._h))

    def free(self):
        if self._h:
            _f_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def bem_server_create(budget_bytes, n_slots):
    return Server(budget_bytes, n_slots)


def bem_server_create_ex(budget_bytes, n_slots, batch_slots):
    return Server(budget_bytes, n_slots, batch_slots)
