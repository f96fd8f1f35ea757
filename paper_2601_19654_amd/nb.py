"""ctypes binding of the C ABI in include/nb.h (argument marshalling only).

Every step of the hot path runs in the HIP library ``libnbody.so``; this module
loads it, converts arguments, and uses PyTorch only for device memory (the
context workspace, device-resident arrays) and for the HIP stream.  There is no
fallback: if the library is missing the import of the functions fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnbody.so")
# tile and algorithm choices per GPU, mode and size class (written by autotune.py)
TUNING_TABLE = os.path.join(_PKG, "tuning.tsv")

NB_OK = 0
NB_E_INVALID = -1
NB_E_NOT_READY = -2
NB_E_HIP = -3
NB_E_NONFINITE = -4
NB_E_CAPACITY = -5
NB_E_KEPLER = -6
NB_E_WORKSPACE = -7
NB_FP64 = 0
NB_FP32C = 1
NB_HELIO = 0
NB_DH = 1
NB_HOST = 0
NB_DEVICE = 1
NB_K_FORCE = 0
NB_K_ENCOUNTER = 1
NB_K_DRIFT = 2
NB_K_STEP = 3
NB_K_FORCE_EVAL = 4
NB_K_FORCE_FUSED = 5


class nb_params(ctypes.Structure):
    _fields_ = [
        ("G", ctypes.c_double), ("n_hill", ctypes.c_double), ("chg_inner", ctypes.c_double),
        ("mode", ctypes.c_int32), ("drag", ctypes.c_int32),
        ("drag_sigma0", ctypes.c_double), ("drag_h", ctypes.c_double),
        ("drag_cd", ctypes.c_double), ("drag_rho_p", ctypes.c_double),
        ("force_jchunk", ctypes.c_int32), ("force_r", ctypes.c_int32),
        ("enc_jchunk", ctypes.c_int32), ("enc_algo", ctypes.c_int32),
        ("step_algo", ctypes.c_int32), ("resolve", ctypes.c_int32),
        ("resolve_threads", ctypes.c_int32), ("force_algo", ctypes.c_int32),
        ("bs_tol", ctypes.c_double), ("autotune_path", ctypes.c_char_p),
        ("force_g", ctypes.c_int32),
    ]


class nb_stats(ctypes.Structure):
    _fields_ = [
        ("total_nce", ctypes.c_int64), ("max_nce", ctypes.c_int32),
        ("overflow_steps", ctypes.c_int32), ("kepler_fail", ctypes.c_int64),
        ("near_pairs", ctypes.c_int64), ("resolved_groups", ctypes.c_int64),
        ("resolved_bodies", ctypes.c_int64), ("max_group", ctypes.c_int32),
        ("bs_fail", ctypes.c_int32),
    ]


class nb_resolve_info(ctypes.Structure):
    _fields_ = [
        ("groups", ctypes.c_int32), ("bodies", ctypes.c_int32), ("max_group", ctypes.c_int32),
        ("failed", ctypes.c_int32), ("max_steps", ctypes.c_int32),
    ]


class nb_event_params(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("r_star", ctypes.c_double), ("r_eject", ctypes.c_double)]


class nb_event_counts(ctypes.Structure):
    _fields_ = [("star", ctypes.c_int32), ("collide", ctypes.c_int32), ("merged", ctypes.c_int32),
                ("ejected", ctypes.c_int32)]


class NbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None

# exported symbol -> (restype, argtypes)
_P, _I, _D, _S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "nb_version": (_I, [_P, _P]),
    "nb_strerror": (ctypes.c_char_p, [_I]),
    "nb_default_params": (None, [_P]),
    "nb_workspace_size": (_I, [_P, _I, _P, _P, _I, _P]),
    "nb_create": (_I, [_P, _I, _P, _P, _I, _P, _S, _P, _P]),
    "nb_last_error": (ctypes.c_char_p, [_P]),
    "nb_upload": (_I, [_P, _P, _P, _P, _P, _I, _I]),
    "nb_download": (_I, [_P, _P, _P, _I, _I]),
    "nb_force": (_I, [_P]),
    "nb_kick": (_I, [_P, _D]),
    "nb_sun_drift": (_I, [_P, _D]),
    "nb_drift": (_I, [_P, _D, _P]),
    "nb_encounters": (_I, [_P, _I, _P, _P, _P, _P, _I]),
    "nb_get_encounters": (_I, [_P, _I, _P, _P, _P, _P, _I]),
    "nb_step": (_I, [_P, _D, _I, _P]),
    "nb_prepare": (_I, [_P, _D, _I]),
    "nb_diagnostics": (_I, [_P, _P, _P, _P, _P]),
    "nb_get_accel": (_I, [_P, _P, _I]),
    "nb_get_rcrit": (_I, [_P, _P, _I]),
    "nb_time_kernel": (_I, [_P, _I, _I, _D, _P]),
    "nb_resolve_host": (_I, [_I, _D, _D, _D, _D, _D, _P, _P, _P, _P, _I, _P, _P, _P, _P, _P, _I, _P]),
    "nb_get_choices": (_I, [_P, _P, _P, _P]),
    "nb_get_params": (_I, [_P, _P, _P]),
    "nb_destroy": (_I, [_P]),
    "nb_events": (_I, [_P, _P, _P, _P, _I]),
    "nb_compact": (_I, [_P, _P, _P, _P, _I]),
    "nb_force_noalloc": (_I, [_P, _I, _D, _P, _P, _P, _P]),
}


def lib():
    """Load libnbody.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built: run __graft_entry__.build()")
        # PyTorch ships its own HIP runtime; load it first so that the library's
        # libamdhip64.so.7 dependency resolves to the same runtime (one runtime
        # per process: streams and device memory are shared with torch).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


NOALLOC_MAX_N = 16384     # include/nb.h: NB_NOALLOC_MAX_N


def force_noalloc(params: nb_params, n: int, m0: float, m, x, a, stream=None, check=True) -> int:
    """nb_force_noalloc on device tensors m[n], x[3, n], a[3, n] (float64,
    contiguous) on the current device; enqueued on `stream` (a torch stream, or
    torch's current stream).  Returns the status (raises on an error when check)."""
    import torch
    for t in (m, x, a):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
            raise ValueError("force_noalloc takes contiguous float64 device tensors")
    if m.numel() < n or x.numel() < 3 * n or a.numel() < 3 * n:
        raise ValueError("force_noalloc: arrays shorter than n")
    s = stream if stream is not None else torch.cuda.current_stream()
    code = lib().nb_force_noalloc(ctypes.byref(params), int(n), float(m0), _addr(m), _addr(x), _addr(a),
                                  ctypes.c_void_p(s.cuda_stream))
    if check and code != NB_OK:
        raise NbError(code, "nb_force_noalloc")
    return code


def strerror(code: int) -> str:
    return lib().nb_strerror(code).decode()


def default_params(**kw) -> nb_params:
    p = nb_params()
    lib().nb_default_params(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _addr(a):
    """Device or host address of a torch tensor or numpy array."""
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Encounters:
    nce: int
    ice: np.ndarray
    jce: np.ndarray
    ce: np.ndarray


def resolve_host(G, m0, m, rc, tau, Q0, V0, ice, jce, Q, V, tol=0.0, inner=0.1, nthreads=0):
    """Host close-encounter resolver on one system's host arrays (n x 3 rows,
    local pair indices).  Returns (Q, V, group, info dict)."""
    m = _f64(m); rc = _f64(rc); n = len(m)
    Q0 = _f64(Q0).reshape(n, 3); V0 = _f64(V0).reshape(n, 3)
    Q = _f64(Q).reshape(n, 3).copy(); V = _f64(V).reshape(n, 3).copy()
    ice = np.ascontiguousarray(ice, dtype=np.int32); jce = np.ascontiguousarray(jce, dtype=np.int32)
    group = np.empty(max(n, 1), np.int32)
    info = nb_resolve_info()
    code = lib().nb_resolve_host(n, float(G), float(m0), float(inner), float(tol), float(tau), _addr(m), _addr(rc),
                                 _addr(Q0), _addr(V0), len(ice), _addr(ice), _addr(jce), _addr(Q), _addr(V),
                                 _addr(group), int(nthreads), ctypes.byref(info))
    if code != NB_OK:
        raise NbError(code, "nb_resolve_host")
    return Q, V, group[:n].copy(), {k: getattr(info, k) for k, _ in nb_resolve_info._fields_}


class Context:
    """One nb_ctx: workspace and stream from PyTorch, every call into libnbody.

    ``off`` are the system offsets (nsys+1); vectors cross the boundary
    plane-major (3, ntot).
    """

    def __init__(self, off, params: nb_params | None = None, enc_cap: int = 1 << 16,
                 stream=None, device=None, tuned: bool = True, nbig=None):
        import torch
        self._torch = torch
        L = lib()
        # a copy: the caller's parameters are not modified
        self.params = nb_params.from_buffer_copy(params) if params is not None else default_params()
        self.off = np.ascontiguousarray(off, dtype=np.int32)
        # per system: the first nbig[s] bodies are big (gravity sources); None = all
        self.nbig = None if nbig is None else np.ascontiguousarray(nbig, dtype=np.int32)
        nbig_p = None if self.nbig is None else _addr(self.nbig)
        # tuned: the library takes the tile and algorithm fields left at 0 from
        # the package's tuning table for this GPU, mode and size class
        self._tuning_path = None
        if tuned and not self.params.autotune_path and os.path.exists(TUNING_TABLE):
            self._tuning_path = TUNING_TABLE.encode()
            self.params.autotune_path = self._tuning_path
        self.nsys = len(self.off) - 1
        self.ntot = int(self.off[-1])
        self.enc_cap = int(enc_cap)
        nbytes = ctypes.c_size_t()
        self._check(L.nb_workspace_size(ctypes.byref(self.params), self.nsys, _addr(self.off), nbig_p,
                                        self.enc_cap, ctypes.byref(nbytes)), "nb_workspace_size")
        self.device = torch.device(device or "cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        self.ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self._check(L.nb_create(ctypes.byref(self.params), self.nsys, _addr(self.off), nbig_p, self.enc_cap,
                                    _addr(self.workspace), nbytes.value,
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self.ctx)),
                        "nb_create")
        # the parameters the library runs with (tuned or default tiles)
        eff, tun = nb_params(), ctypes.c_int32()
        self._check(L.nb_get_params(self.ctx, ctypes.byref(eff), ctypes.byref(tun)), "nb_get_params")
        self.params = eff
        self.tiles = "tuned" if tun.value else "library defaults"

    def _check(self, code, what, allow=()):
        if code != NB_OK and code not in allow:
            msg = what
            if getattr(self, "ctx", None):
                detail = lib().nb_last_error(self.ctx)
                if detail:
                    msg += ": " + detail.decode()
            raise NbError(code, f"{msg}: {strerror(code)}")
        return code

    # ------------------------------------------------------------ state
    def upload(self, m0, m, x, v, frame=NB_HELIO):
        """x, v: (ntot, 3) or (3, ntot) host arrays, or (3, ntot) device tensors."""
        torch = self._torch
        if isinstance(x, torch.Tensor) and x.is_cuda:
            args = [t.contiguous() for t in (m0, m, x, v)]
            where = NB_DEVICE
        else:
            x = np.asarray(x); v = np.asarray(v)
            if x.shape == (self.ntot, 3) and self.ntot != 3:
                x, v = x.T, v.T
            args = [_f64(m0), _f64(m), _f64(x), _f64(v)]
            where = NB_HOST
        self._keep = args
        self._check(lib().nb_upload(self.ctx, *[_addr(a) for a in args], frame, where), "nb_upload")

    def download(self, frame=NB_HELIO):
        x = np.empty((3, self.ntot)); v = np.empty((3, self.ntot))
        self._check(lib().nb_download(self.ctx, _addr(x), _addr(v), frame, NB_HOST), "nb_download")
        return x.T.copy(), v.T.copy()

    def download_device(self, x, v, frame=NB_HELIO):
        self._check(lib().nb_download(self.ctx, _addr(x), _addr(v), frame, NB_DEVICE), "nb_download")

    # ------------------------------------------------------------ sub-steps
    def force(self):
        self._check(lib().nb_force(self.ctx), "nb_force")

    def kick(self, h):
        self._check(lib().nb_kick(self.ctx, float(h)), "nb_kick")

    def sun_drift(self, h):
        self._check(lib().nb_sun_drift(self.ctx, float(h)), "nb_sun_drift")

    def drift(self, dt, allow_fail=False):
        nf = ctypes.c_int()
        self._check(lib().nb_drift(self.ctx, float(dt), ctypes.byref(nf)), "nb_drift",
                    allow=(NB_E_KEPLER,) if allow_fail else ())
        return nf.value

    def _enc(self, fn, cap, allow_overflow):
        cap = self.enc_cap if cap is None else cap
        n = ctypes.c_int()
        ice = np.zeros(max(cap, 1), np.int32); jce = np.zeros(max(cap, 1), np.int32)
        ce = np.zeros(max(self.ntot, 1), np.int32)
        self._check(fn(self.ctx, cap, ctypes.byref(n), _addr(ice), _addr(jce), _addr(ce), NB_HOST),
                    fn.__name__, allow=(NB_E_CAPACITY,) if allow_overflow else ())
        k = min(n.value, cap)
        return Encounters(n.value, ice[:k], jce[:k], ce[:self.ntot])

    def encounters(self, cap=None, allow_overflow=False):
        return self._enc(lib().nb_encounters, cap, allow_overflow)

    def last_encounters(self, cap=None, allow_overflow=False):
        return self._enc(lib().nb_get_encounters, cap, allow_overflow)

    def step(self, dt, nsteps=1, allow=()):
        st = nb_stats()
        self._check(lib().nb_step(self.ctx, float(dt), int(nsteps), ctypes.byref(st)), "nb_step",
                    allow=allow)
        return {k: getattr(st, k) for k, _ in nb_stats._fields_}

    def prepare(self, dt, nsteps):
        """Capture the HIP graphs a step(dt, nsteps) call replays, running nothing."""
        self._check(lib().nb_prepare(self.ctx, float(dt), int(nsteps)), "nb_prepare")

    def step_async(self, dt, nsteps=1):
        """nb_step without the statistics argument (still synchronizes at the end)."""
        return self._check(lib().nb_step(self.ctx, float(dt), int(nsteps), None), "nb_step",
                           allow=(NB_E_CAPACITY, NB_E_KEPLER))

    # ------------------------------------------------------------ events
    def events(self, rho, r_star=0.0, r_eject=0.0, allow_overflow=False):
        """Star impacts, collisions and ejections of the last step; returns
        (counts dict, lost flags per body)."""
        ep = nb_event_params(float(rho), float(r_star), float(r_eject))
        cnt = nb_event_counts()
        lost = np.zeros(max(self.ntot, 1), np.int32)
        self._check(lib().nb_events(self.ctx, ctypes.byref(ep), ctypes.byref(cnt), _addr(lost), NB_HOST),
                    "nb_events", allow=(NB_E_CAPACITY,) if allow_overflow else ())
        return {k: getattr(cnt, k) for k, _ in nb_event_counts._fields_}, lost[:self.ntot]

    def compact(self):
        """Remove the lost bodies; returns the old index of every kept body and
        updates off, ntot and nbig."""
        off = np.zeros(self.nsys + 1, np.int32)
        nbig = np.zeros(max(self.nsys, 1), np.int32)
        idx = np.zeros(max(self.ntot, 1), np.int32)
        self._check(lib().nb_compact(self.ctx, _addr(off), _addr(nbig), _addr(idx), NB_HOST), "nb_compact")
        self.off = off
        self.ntot = int(off[-1])
        if self.nbig is not None:
            self.nbig = nbig[:self.nsys].copy()
        return idx[:self.ntot].copy()

    # ------------------------------------------------------------ outputs
    def diagnostics(self):
        E = np.empty(self.nsys); EK = np.empty(self.nsys)
        L = np.empty((self.nsys, 3)); P = np.empty((self.nsys, 3))
        self._check(lib().nb_diagnostics(self.ctx, _addr(E), _addr(EK), _addr(L), _addr(P)),
                    "nb_diagnostics")
        return {"E": E, "EK": EK, "L": L, "P": P}

    def accel(self):
        a = np.empty((3, self.ntot))
        self._check(lib().nb_get_accel(self.ctx, _addr(a), NB_HOST), "nb_get_accel")
        return a.T.copy()

    def rcrit(self):
        rc = np.empty(self.ntot)
        self._check(lib().nb_get_rcrit(self.ctx, _addr(rc), NB_HOST), "nb_get_rcrit")
        return rc

    def time_kernel(self, which, reps=10, dt=0.0):
        """Mean milliseconds per launch of one kernel (HIP events on this stream)."""
        ms = ctypes.c_double()
        self._check(lib().nb_time_kernel(self.ctx, int(which), int(reps), float(dt), ctypes.byref(ms)),
                    "nb_time_kernel")
        return ms.value

    def choices(self):
        """Resolved algorithms: force (1 ordered, 2 symmetric, 3 few sources),
        encounter check (1 direct, 2 sorted), step launch (1 per phase, 2 persistent),
        and the symmetric force's super-tile width."""
        f, e, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self._check(lib().nb_get_choices(self.ctx, ctypes.byref(f), ctypes.byref(e), ctypes.byref(st)),
                    "nb_get_choices")
        return {"force_algo": f.value, "enc_algo": e.value, "step_algo": st.value,
                "force_g": int(self.params.force_g)}

    def close(self):
        if getattr(self, "ctx", None):
            lib().nb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def version():
    a, b = ctypes.c_int(), ctypes.c_int()
    lib().nb_version(ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value
