"""Python access to the plain FP64 CPU oracle (``pdbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.  It does not
import the product package.

The oracle keeps its state as f[ir][jt][q] (array of structures) with
q = 0 for the rest particle and q = 1 + 8(k-1) + i for speed k = 1..4 and
direction i = 0..7 (Sec. II.B of Lin, Xu, Zhang, Li, arXiv:1308.0653).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdbm_oracle.c")
LIB = {"double": os.path.join(HERE, "liboracle.so"),
       "long double": os.path.join(HERE, "liboracle_ld.so")}
NQ = 33


def build(force: bool = True) -> None:
    """Compile both oracle variants with gcc (IEEE order kept: no contraction,
    no fast-math)."""
    for real, out in LIB.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        tmp = out + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-shared", "-fPIC", f"-DORA_REAL={real}", SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


class Params(C.Structure):
    _fields_ = [("nr", C.c_int32), ("ntheta", C.c_int32), ("sector", C.c_int32),
                ("m", C.c_int32), ("n", C.c_int32), ("pad_", C.c_int32),
                ("r_min", C.c_double), ("r_max", C.c_double), ("dt", C.c_double),
                ("tau", C.c_double), ("w1", C.c_double), ("w2", C.c_double),
                ("Q", C.c_double), ("T_th", C.c_double)]


_libs: dict = {}


def lib(real: str = "double"):
    if real not in _libs:
        path = LIB[real]
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(SRC):
            build(force=False)
        L = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        L.ora_create.restype = vp
        L.ora_create.argtypes = [C.POINTER(Params)]
        L.ora_destroy.argtypes = [vp]
        L.ora_init_ic.argtypes = [vp, C.c_double, dp, dp, C.c_double, C.c_uint64]
        L.ora_init_fields.argtypes = [vp, dp]
        L.ora_set_state.argtypes = [vp, dp, dp, C.c_longlong]
        L.ora_get_state.argtypes = [vp, dp, dp]
        L.ora_step.argtypes = [vp, C.c_longlong]
        L.ora_step_count.argtypes = [vp]
        L.ora_step_count.restype = C.c_longlong
        L.ora_set_tau.argtypes = [vp, C.c_void_p]
        L.ora_fields.argtypes = [vp, dp]
        L.ora_diag.argtypes = [vp, dp, np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")]
        L.ora_weights.argtypes = [C.c_double, dp]
        L.ora_velocities.argtypes = [C.c_double, dp, dp]
        L.ora_equilibrium.argtypes = [C.c_double] * 5 + [dp]
        L.ora_moments.argtypes = [dp, C.c_double, dp]
        L.ora_collide.argtypes = [C.POINTER(Params), dp, C.c_double, C.c_double, dp, dp]
        L.ora_cochran.argtypes = [C.c_double] * 4
        L.ora_cochran.restype = C.c_double
        L.ora_noneq.argtypes = [vp, dp]
        L.ora_central_moments.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp]
        L.ora_splitmix64.argtypes = [C.c_uint64]
        L.ora_splitmix64.restype = C.c_uint64
        L.ora_real_bytes.restype = C.c_int
        _libs[real] = L
    return _libs[real]


def make_params(nr, ntheta, r_min, r_max, dt, tau, w1=0.0, w2=0.0, m=1, n=1,
                Q=1.0, T_th=1.1, sector=8) -> Params:
    return Params(int(nr), int(ntheta), int(sector), int(m), int(n), 0,
                  float(r_min), float(r_max), float(dt), float(tau), float(w1),
                  float(w2), float(Q), float(T_th))


# ------------------------------------------------------------ per-cell ----

def weights(T: float) -> np.ndarray:
    out = np.zeros(5)
    lib().ora_weights(float(T), out)
    return out


def velocities(theta: float):
    vr, vt = np.zeros(NQ), np.zeros(NQ)
    lib().ora_velocities(float(theta), vr, vt)
    return vr, vt


def equilibrium(rho, ur, ut, T, theta) -> np.ndarray:
    out = np.zeros(NQ)
    lib().ora_equilibrium(float(rho), float(ur), float(ut), float(T), float(theta), out)
    return out


def moments(f, theta):
    out = np.zeros(4)
    lib().ora_moments(np.ascontiguousarray(f, dtype=np.float64), float(theta), out)
    return out  # rho, u_r, u_theta, T


def collide(params: Params, f, lam, theta):
    out, info = np.zeros(NQ), np.zeros(7)
    lib().ora_collide(C.byref(params), np.ascontiguousarray(f, dtype=np.float64),
                      float(lam), float(theta), out, info)
    return out, info  # info = rho, u_r, u_theta, T, a, b, reacting


def cochran(lam, a, b, dt) -> float:
    return lib().ora_cochran(float(lam), float(a), float(b), float(dt))


NONEQ_NAMES = ("D2_rr", "D2_rt", "D2_tt", "D3_rrr", "D3_rrt", "D3_rtt", "D3_ttt",
               "D31_r", "D31_t", "D42_rr", "D42_rt", "D42_tt")


def central_moments(g, theta, ur, ut) -> np.ndarray:
    """M*_2, M*_3, M*_{3,1}, M*_{4,2} of g about (u_r, u_theta), in the order of
    NONEQ_NAMES (Sec. II.E)."""
    out = np.zeros(12)
    lib().ora_central_moments(np.ascontiguousarray(g, dtype=np.float64), float(theta), float(ur), float(ut), out)
    return out


def splitmix64(x: int) -> int:
    return int(lib().ora_splitmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


# --------------------------------------------------------------- state ----

class Solver:
    """One oracle solve.  ``real`` selects double or long double arithmetic."""

    def __init__(self, params: Params, real: str = "double"):
        self.L = lib(real)
        self.p = params
        self.h = self.L.ora_create(C.byref(params))
        if not self.h:
            raise ValueError("invalid oracle parameters")

    def close(self):
        if self.h:
            self.L.ora_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def shape(self):
        return (self.p.nr, self.p.ntheta)

    def init_ic(self, r_split, inner, outer, p_noise=0.0, seed=0):
        self.L.ora_init_ic(self.h, float(r_split), np.asarray(inner, dtype=np.float64),
                           np.asarray(outer, dtype=np.float64), float(p_noise),
                           int(seed) & 0xFFFFFFFFFFFFFFFF)

    def init_fields(self, fields):
        """fields: [5][nr][ntheta] = rho, T, u_r, u_theta, lambda."""
        self.L.ora_init_fields(self.h, np.ascontiguousarray(fields, dtype=np.float64))

    def set_state(self, f, lam, step=0):
        nr, nt = self.shape
        self.L.ora_set_state(self.h, np.ascontiguousarray(f, dtype=np.float64).reshape(nr, nt, NQ),
                             np.ascontiguousarray(lam, dtype=np.float64).reshape(nr, nt), int(step))

    def get_state(self):
        nr, nt = self.shape
        f, lam = np.zeros((nr, nt, NQ)), np.zeros((nr, nt))
        self.L.ora_get_state(self.h, f, lam)
        return f, lam

    def set_tau(self, tau):
        """Per-cell relaxation time [nr][ntheta] (Sec. IV, point (ii)), or
        None for the parameters' tau in every cell."""
        if tau is None:
            self.L.ora_set_tau(self.h, None)
            return
        t = np.ascontiguousarray(tau, dtype=np.float64).reshape(self.shape)
        self.L.ora_set_tau(self.h, t.ctypes.data_as(C.c_void_p))

    def step(self, n=1):
        self.L.ora_step(self.h, int(n))

    @property
    def step_count(self):
        return self.L.ora_step_count(self.h)

    def fields(self) -> np.ndarray:
        """[6][nr][ntheta] = rho, u_r, u_theta, T, p, lambda."""
        nr, nt = self.shape
        out = np.zeros((6, nr, nt))
        self.L.ora_fields(self.h, out)
        return out

    def noneq(self) -> np.ndarray:
        """[12][nr][ntheta] non-equilibrium measures Delta*_m (Sec. II.E), in
        the order of NONEQ_NAMES."""
        nr, nt = self.shape
        out = np.zeros((12, nr, nt))
        self.L.ora_noneq(self.h, out)
        return out

    def diag(self):
        out, cnt = np.zeros(3), np.zeros(2, dtype=np.int64)
        self.L.ora_diag(self.h, out, cnt)
        return {"mass": out[0], "energy": out[1], "chem": out[2],
                "n_nonfinite": int(cnt[0]), "n_nonphys": int(cnt[1])}
