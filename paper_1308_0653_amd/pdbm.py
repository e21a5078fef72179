"""ctypes binding of libpdbm (include/pdbm.h): argument marshalling only.

Every function keeps its C name.  All numerical work runs in the HIP kernels
of libpdbm.so; this module never computes a step itself and raises if the
library is missing or has no gfx950 device to run on.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

LIB_PATH = _build.LIB

PDBM_OK, PDBM_EINVAL, PDBM_ECFL, PDBM_ENOMEM, PDBM_EHIP = 0, -1, -2, -3, -4
PDBM_EAGAIN, PDBM_ENOENT, PDBM_ENONPHYS, PDBM_ENOSYS = -5, -6, -7, -8
PDBM_FP64, PDBM_FP32 = 0, 1
PDBM_QUEUED, PDBM_RUNNING, PDBM_DONE, PDBM_FAILED = 0, 1, 2, 3
PDBM_ALLOW_CFL = 1
PDBM_TAU_FIELD = 2
PDBM_SCRATCH_BYTES = 16 << 20
NQ = 33
# components of pdbm_noneq's output (Sec. II.E), in order
NONEQ_NAMES = ("D2_rr", "D2_rt", "D2_tt", "D3_rrr", "D3_rrt", "D3_rtt", "D3_ttt",
               "D31_r", "D31_t", "D42_rr", "D42_rt", "D42_tt")
PDBM_NONEQ_N = len(NONEQ_NAMES)


class pdbm_params(C.Structure):
    _fields_ = [("nr", C.c_int32), ("ntheta", C.c_int32), ("sector", C.c_int32),
                ("precision", C.c_int32), ("m", C.c_int32), ("n", C.c_int32),
                ("diag_every", C.c_int32), ("flags", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double), ("dt", C.c_double),
                ("tau", C.c_double), ("w1", C.c_double), ("w2", C.c_double),
                ("Q", C.c_double), ("T_th", C.c_double)]


class pdbm_ic(C.Structure):
    _fields_ = [("r_split", C.c_double), ("inner", C.c_double * 5), ("outer", C.c_double * 5),
                ("p_noise", C.c_double), ("seed", C.c_uint64)]


class pdbm_diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("mass", C.c_double), ("energy", C.c_double),
                ("chem", C.c_double), ("n_nonfinite", C.c_int64), ("n_nonphys", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pdbm_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("queued", C.c_int64), ("running", C.c_int64), ("done", C.c_int64),
                ("failed", C.c_int64), ("steps_launched", C.c_int64), ("hbm_in_use", C.c_size_t),
                ("hbm_cap", C.c_size_t), ("cell_updates", C.c_double), ("elapsed", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


PDBM_KEEP_FIELDS = 1


class PdbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def lib():
    """Loads libpdbm.so (building it first only if it does not exist)."""
    global _lib
    if _lib is None:
        # Bring in torch's HIP runtime first when torch is installed, so that
        # the process holds one HIP runtime and torch streams and device
        # memory are valid handles for the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            _build.build()
        L = C.CDLL(LIB_PATH)
        vp, dp = C.c_void_p, C.POINTER(C.c_double)
        sig = {
            "pdbm_strerror": (C.c_char_p, [C.c_int]),
            "pdbm_last_error": (C.c_char_p, []),
            "pdbm_version": (C.c_int, []),
            "pdbm_validate": (C.c_int, [C.POINTER(pdbm_params), C.POINTER(pdbm_ic), dp]),
            "pdbm_state_bytes": (C.c_int, [C.POINTER(pdbm_params), C.POINTER(C.c_size_t)]),
            "pdbm_fk_matrix": (C.c_int, [dp]),
            "pdbm_create": (C.c_int, [C.POINTER(pdbm_params), C.POINTER(pdbm_ic), vp, C.c_size_t, vp,
                                      C.POINTER(vp)]),
            "pdbm_create_noalloc": (C.c_int, [C.POINTER(pdbm_params), C.POINTER(pdbm_ic), vp,
                                              C.POINTER(C.c_size_t), vp, C.POINTER(vp)]),
            "pdbm_destroy": (None, [vp]),
            "pdbm_set_fields": (C.c_int, [vp, dp]),
            "pdbm_set_tau": (C.c_int, [vp, dp]),
            "pdbm_set_tau_async": (C.c_int, [vp, vp]),
            "pdbm_step": (C.c_int, [vp, C.c_int64]),
            "pdbm_step_count": (C.c_int64, [vp]),
            "pdbm_moments": (C.c_int, [vp, dp, C.POINTER(pdbm_diag)]),
            "pdbm_moments_async": (C.c_int, [vp, vp]),
            "pdbm_noneq": (C.c_int, [vp, dp]),
            "pdbm_noneq_async": (C.c_int, [vp, vp]),
            "pdbm_batch_noneq": (C.c_int, [vp, C.c_int32, dp]),
            "pdbm_diag_history": (C.c_int, [vp, C.POINTER(pdbm_diag), C.c_int32, C.POINTER(C.c_int32)]),
            "pdbm_read_f": (C.c_int, [vp, dp, dp]),
            "pdbm_write_f": (C.c_int, [vp, dp, dp, C.c_int64]),
            "pdbm_get_state": (C.c_int, [vp, vp, C.POINTER(C.c_size_t)]),
            "pdbm_set_state": (C.c_int, [vp, vp, C.c_size_t]),
            "pdbm_batch_create": (C.c_int, [C.c_int32, C.POINTER(pdbm_params), C.POINTER(pdbm_ic), C.c_int32, vp,
                                            C.POINTER(vp)]),
            "pdbm_batch_destroy": (None, [vp]),
            "pdbm_batch_step": (C.c_int, [vp, C.c_int64]),
            "pdbm_batch_step_count": (C.c_int64, [vp, C.c_int32]),
            "pdbm_batch_moments": (C.c_int, [vp, C.c_int32, dp, C.POINTER(pdbm_diag)]),
            "pdbm_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.c_int32, vp, C.POINTER(vp)]),
            "pdbm_server_destroy": (None, [vp]),
            "pdbm_submit": (C.c_int, [vp, C.POINTER(pdbm_params), C.POINTER(pdbm_ic), C.c_int64, C.c_uint32,
                                      C.POINTER(C.c_uint64)]),
            "pdbm_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(C.c_int32), dp, C.POINTER(pdbm_diag)]),
            "pdbm_request_times": (C.c_int, [vp, C.c_uint64, dp]),
            "pdbm_release": (C.c_int, [vp, C.c_uint64]),
            "pdbm_server_wait": (C.c_int, [vp, C.c_double]),
            "pdbm_server_get_stats": (C.c_int, [vp, C.POINTER(pdbm_server_stats)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc != PDBM_OK:
        L = lib()
        raise PdbmError(rc, f"{L.pdbm_strerror(rc).decode()}: {L.pdbm_last_error().decode()}")
    return rc


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(nr, ntheta, r_min, r_max, dt, tau, w1=0.0, w2=0.0, m=1, n=1, Q=1.0, T_th=1.1,
                sector=8, precision=PDBM_FP64, diag_every=0, flags=0) -> pdbm_params:
    return pdbm_params(int(nr), int(ntheta), int(sector), int(precision), int(m), int(n), int(diag_every),
                       int(flags), float(r_min), float(r_max), float(dt), float(tau), float(w1), float(w2),
                       float(Q), float(T_th))


def make_ic(r_split, inner, outer, p_noise=0.0, seed=0) -> pdbm_ic:
    return pdbm_ic(float(r_split), (C.c_double * 5)(*map(float, inner)), (C.c_double * 5)(*map(float, outer)),
                   float(p_noise), int(seed) & 0xFFFFFFFFFFFFFFFF)


def _stream_handle(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream


# ------------------------------------------------------------ C names ----

def pdbm_validate(params: pdbm_params, ic: pdbm_ic | None = None) -> float:
    cfl = C.c_double(0.0)
    _check(lib().pdbm_validate(C.byref(params), C.byref(ic) if ic is not None else None, C.byref(cfl)))
    return cfl.value


def pdbm_state_bytes(params: pdbm_params) -> int:
    n = C.c_size_t(0)
    _check(lib().pdbm_state_bytes(C.byref(params), C.byref(n)))
    return n.value


def pdbm_fk_matrix() -> np.ndarray:
    A = np.zeros(16)
    _check(lib().pdbm_fk_matrix(_dptr(A)))
    return A.reshape(4, 4)


def pdbm_create(params: pdbm_params, ic: pdbm_ic | None = None, workspace=None, stream=None) -> "Solver":
    return Solver(params, ic, workspace=workspace, stream=stream)


def pdbm_noalloc_state_bytes(params: pdbm_params) -> int:
    """Bytes of the state buffer pdbm_create_noalloc needs (its size query)."""
    n = C.c_size_t(0)
    _check(lib().pdbm_create_noalloc(C.byref(params), None, None, C.byref(n), None, None))
    return n.value


def pdbm_create_noalloc(params: pdbm_params, ic: pdbm_ic | None, state, stream=None) -> "Solver":
    """A solve whose state lives in the caller's device tensor `state` and
    whose other device memory is the library's static scratch."""
    return Solver(params, ic, workspace=state, stream=stream, noalloc=True)


class Solver:
    """Handle of one solve; methods are the pdbm_* calls on it."""

    def __init__(self, params: pdbm_params, ic: pdbm_ic | None = None, workspace=None, stream=None,
                 noalloc: bool = False):
        self.L = lib()
        self.params = params
        self.nr, self.nt = params.nr, params.ntheta
        self.h = C.c_void_p()
        ws_ptr, ws_bytes = None, 0
        self._ws = workspace  # keep the caller's buffer (e.g. a torch tensor) alive
        if workspace is not None:
            ws_ptr = C.c_void_p(int(workspace.data_ptr()))
            ws_bytes = workspace.numel() * workspace.element_size()
        self.stream = _stream_handle(stream)
        icp = C.byref(ic) if ic is not None else None
        if noalloc:
            assert workspace is not None, "pdbm_create_noalloc needs the caller's state buffer"
            n = C.c_size_t(ws_bytes)
            _check(self.L.pdbm_create_noalloc(C.byref(params), icp, ws_ptr, C.byref(n), C.c_void_p(self.stream),
                                              C.byref(self.h)))
        else:
            _check(self.L.pdbm_create(C.byref(params), icp, ws_ptr, ws_bytes, C.c_void_p(self.stream),
                                      C.byref(self.h)))

    def close(self):
        if self.h:
            self.L.pdbm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def pdbm_set_tau(self, tau):
        """Per-cell relaxation time [nr][ntheta] (host array), or None for the
        parameters' tau everywhere (needs PDBM_TAU_FIELD)."""
        if tau is None:
            _check(self.L.pdbm_set_tau(self.h, None))
            return
        a = np.ascontiguousarray(tau, dtype=np.float64)
        assert a.shape == (self.nr, self.nt)
        _check(self.L.pdbm_set_tau(self.h, _dptr(a)))

    set_tau = pdbm_set_tau

    def pdbm_set_tau_async(self, tau_tensor):
        """As pdbm_set_tau from a float64 device tensor [nr][ntheta], enqueued
        on the solver's stream."""
        assert tau_tensor.is_cuda and tau_tensor.is_contiguous() and tau_tensor.numel() == self.nr * self.nt
        _check(self.L.pdbm_set_tau_async(self.h, C.c_void_p(int(tau_tensor.data_ptr()))))

    set_tau_async = pdbm_set_tau_async

    def pdbm_step(self, nsteps: int = 1):
        _check(self.L.pdbm_step(self.h, int(nsteps)))

    step = pdbm_step

    @property
    def step_count(self) -> int:
        return self.L.pdbm_step_count(self.h)

    def pdbm_set_fields(self, fields: np.ndarray):
        a = np.ascontiguousarray(fields, dtype=np.float64)
        assert a.shape == (5, self.nr, self.nt)
        _check(self.L.pdbm_set_fields(self.h, _dptr(a)))

    set_fields = pdbm_set_fields

    def pdbm_moments(self, check: bool = True):
        """Returns (fields [6][nr][ntheta] = rho, u_r, u_theta, T, p, lambda;
        drift report dict)."""
        out = np.empty((6, self.nr, self.nt))
        d = pdbm_diag()
        rc = self.L.pdbm_moments(self.h, _dptr(out), C.byref(d))
        if rc != PDBM_ENONPHYS or check:
            _check(rc)
        return out, d.as_dict()

    moments = pdbm_moments

    def pdbm_moments_async(self, out_tensor):
        """Enqueues the fields into a caller-owned float64 device tensor of
        shape [6][nr][ntheta]."""
        assert out_tensor.is_cuda and out_tensor.is_contiguous() and out_tensor.numel() == 6 * self.nr * self.nt
        _check(self.L.pdbm_moments_async(self.h, C.c_void_p(int(out_tensor.data_ptr()))))

    moments_async = pdbm_moments_async

    def pdbm_noneq(self) -> np.ndarray:
        """Non-equilibrium measures [12][nr][ntheta] (Sec. II.E), components
        in the order of NONEQ_NAMES."""
        out = np.empty((PDBM_NONEQ_N, self.nr, self.nt))
        _check(self.L.pdbm_noneq(self.h, _dptr(out)))
        return out

    noneq = pdbm_noneq

    def pdbm_noneq_async(self, out_tensor):
        """Enqueues the non-equilibrium measures into a caller-owned float64
        device tensor of shape [12][nr][ntheta]."""
        assert (out_tensor.is_cuda and out_tensor.is_contiguous()
                and out_tensor.numel() == PDBM_NONEQ_N * self.nr * self.nt)
        _check(self.L.pdbm_noneq_async(self.h, C.c_void_p(int(out_tensor.data_ptr()))))

    noneq_async = pdbm_noneq_async

    def pdbm_diag_history(self, cap: int = 4096):
        buf = (pdbm_diag * cap)()
        n = C.c_int32(0)
        _check(self.L.pdbm_diag_history(self.h, buf, cap, C.byref(n)))
        return [buf[i].as_dict() for i in range(n.value)]

    diag_history = pdbm_diag_history

    def pdbm_read_f(self):
        f = np.empty((NQ, self.nr, self.nt))
        lam = np.empty((self.nr, self.nt))
        _check(self.L.pdbm_read_f(self.h, _dptr(f), _dptr(lam)))
        return f, lam

    read_f = pdbm_read_f

    def pdbm_write_f(self, f: np.ndarray, lam: np.ndarray, step: int = 0):
        fa = np.ascontiguousarray(f, dtype=np.float64)
        la = np.ascontiguousarray(lam, dtype=np.float64)
        assert fa.shape == (NQ, self.nr, self.nt) and la.shape == (self.nr, self.nt)
        _check(self.L.pdbm_write_f(self.h, _dptr(fa), _dptr(la), int(step)))

    write_f = pdbm_write_f

    def pdbm_get_state(self) -> bytes:
        n = C.c_size_t(0)
        _check(self.L.pdbm_get_state(self.h, None, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        _check(self.L.pdbm_get_state(self.h, buf, C.byref(n)))
        return buf.raw[: n.value]

    get_state = pdbm_get_state

    def pdbm_set_state(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(self.L.pdbm_set_state(self.h, buf, len(blob)))

    set_state = pdbm_set_state


class Batch:
    """Handle of a packed batch of independent solves (pdbm_batch_*)."""

    def __init__(self, params: list, ics: list | None = None, chunk_steps: int = 0, stream=None):
        self.L = lib()
        n = len(params)
        self.shapes = [(p.nr, p.ntheta) for p in params]
        P = (pdbm_params * n)(*params)
        I = (pdbm_ic * n)(*ics) if ics is not None else None
        self.h = C.c_void_p()
        _check(self.L.pdbm_batch_create(n, P, I, int(chunk_steps), C.c_void_p(_stream_handle(stream)),
                                        C.byref(self.h)))

    def close(self):
        if self.h:
            self.L.pdbm_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pdbm_batch_step(self, nsteps: int = 1):
        _check(self.L.pdbm_batch_step(self.h, int(nsteps)))

    step = pdbm_batch_step

    def step_count(self, i: int) -> int:
        return self.L.pdbm_batch_step_count(self.h, int(i))

    def pdbm_batch_moments(self, i: int, check: bool = True):
        nr, nt = self.shapes[i]
        out = np.empty((6, nr, nt))
        d = pdbm_diag()
        rc = self.L.pdbm_batch_moments(self.h, int(i), _dptr(out), C.byref(d))
        if rc != PDBM_ENONPHYS or check:
            _check(rc)
        return out, d.as_dict()

    moments = pdbm_batch_moments

    def pdbm_batch_noneq(self, i: int) -> np.ndarray:
        nr, nt = self.shapes[i]
        out = np.empty((PDBM_NONEQ_N, nr, nt))
        _check(self.L.pdbm_batch_noneq(self.h, int(i), _dptr(out)))
        return out

    noneq = pdbm_batch_noneq


class Server:
    """Handle of a continuous-batching request server (pdbm_server_*)."""

    def __init__(self, hbm_cap_bytes: int, max_slots: int = 64, chunk_steps: int = 50, stream=None):
        self.L = lib()
        self.h = C.c_void_p()
        self.shapes = {}
        _check(self.L.pdbm_server_create(int(hbm_cap_bytes), int(max_slots), int(chunk_steps),
                                         C.c_void_p(_stream_handle(stream)), C.byref(self.h)))

    def close(self):
        if self.h:
            self.L.pdbm_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pdbm_submit(self, params: pdbm_params, ic: pdbm_ic, nsteps: int, keep_fields: bool = False) -> int:
        rid = C.c_uint64(0)
        _check(self.L.pdbm_submit(self.h, C.byref(params), C.byref(ic), int(nsteps),
                                  PDBM_KEEP_FIELDS if keep_fields else 0, C.byref(rid)))
        self.shapes[rid.value] = (params.nr, params.ntheta, keep_fields)
        return rid.value

    submit = pdbm_submit

    def pdbm_poll(self, rid: int, fields: bool = False):
        """Returns (state, fields or None, drift report or None); state is
        PDBM_QUEUED / RUNNING / DONE / FAILED."""
        st = C.c_int32(-1)
        d = pdbm_diag()
        out = None
        nr, nt, kept = self.shapes.get(rid, (0, 0, False))
        if fields and kept:
            out = np.empty((6, nr, nt))
        rc = self.L.pdbm_poll(self.h, C.c_uint64(rid), C.byref(st), _dptr(out) if out is not None else None,
                              C.byref(d))
        if rc == PDBM_EAGAIN:
            return st.value, None, None
        _check(rc)
        return st.value, out, d.as_dict()

    poll = pdbm_poll

    def times(self, rid: int):
        t = np.zeros(3)
        _check(self.L.pdbm_request_times(self.h, C.c_uint64(rid), _dptr(t)))
        return t

    def release(self, rid: int):
        _check(self.L.pdbm_release(self.h, C.c_uint64(rid)))
        self.shapes.pop(rid, None)

    def wait(self, timeout_s: float = -1.0) -> bool:
        rc = self.L.pdbm_server_wait(self.h, float(timeout_s))
        if rc == PDBM_EAGAIN:
            return False
        _check(rc)
        return True

    def stats(self) -> dict:
        st = pdbm_server_stats()
        _check(self.L.pdbm_server_get_stats(self.h, C.byref(st)))
        return st.as_dict()
