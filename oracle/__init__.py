"""Oracle for the WENO-TT hot path: plain, slow, obviously correct CPU code.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package; the
product library never does, and shares no code with it.

Contents
  * ``weno_oracle.c`` (wrapped here): the dense FD WENO5-JS + global Lax-Friedrichs +
    SSP-RK3 scheme for the Euler equations and two scalar laws (Sec. 2, Sec. 4.4, Sec. 5.1-5.2).
  * ``riemann.py``: the exact solution of the 1D Riemann problem (Sod, Sec. 5.5).
  * ``tt_ref.py``: tensor-train definitions (eq. TT_def), TT-SVD and the rounding bound
    (Sec. 3.1-3.2) and a brute-force maxvol dominance check (Sec. 3.3), in NumPy FP64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_SRC = os.path.join(_HERE, "weno_oracle.c")

OK, EINVAL, ENOMEM, ENONPHYS = 0, -1, -2, -5
BC_PERIODIC, BC_TRANSMISSIVE, BC_SYMMETRY, BC_INFLOW = 0, 1, 2, 3
EULER, LINADV, BURGERS = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int), ("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3),
                ("h", ctypes.c_double * 3), ("gamma", ctypes.c_double), ("bc", (ctypes.c_int * 2) * 3),
                ("inflow", ((ctypes.c_double * 5) * 2) * 3)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.or_alpha.argtypes = [P, dp, dp]
        lib.or_interface_flux.argtypes = [P, ctypes.c_double, dp, ctypes.c_int, dp]
        lib.or_rhs.argtypes = [P, ctypes.c_double, dp, dp]
        lib.or_rhs_naive.argtypes = [P, ctypes.c_double, dp, dp]
        lib.or_ssprk3.argtypes = [P, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.or_run.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp,
                               ctypes.POINTER(ctypes.c_int64)]
        lib.or_inflow_conserved.argtypes = [P, dp, dp]
        lib.or_inflow_conserved.restype = None
        for f in (lib.or_alpha, lib.or_interface_flux, lib.or_rhs, lib.or_rhs_naive, lib.or_ssprk3, lib.or_run):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__({ENONPHYS: "non-physical state (rho<=0 or p<=0)", ENOMEM: "out of memory",
                          EINVAL: "invalid argument"}.get(status, f"status {status}"))
        self.status = status


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Problem:
    """A dense problem on a uniform cell-centred grid.

    ``n`` are the interior cells per dimension, ``lo``/``hi`` the domain box, ``bc`` one
    boundary type per dimension, or a (low, high) pair of them (periodic only in pairs).
    ``inflow`` maps (dimension, side) of each BC_INFLOW side to its primitive state
    (rho, u_1..u_ndim, p) for the Euler law or (u,) for a scalar law (Sec. 4.5.2).
    """

    def __init__(self, n, lo, hi, bc, gamma: float = 1.4, model: int = EULER, inflow=None):
        self.ndim = len(n)
        self.n = tuple(int(v) for v in n)
        self.lo = tuple(float(v) for v in lo)
        self.hi = tuple(float(v) for v in hi)
        self.h = tuple((b - a) / m for a, b, m in zip(self.lo, self.hi, self.n))
        self.bc = tuple((int(b), int(b)) if np.ndim(b) == 0 else (int(b[0]), int(b[1])) for b in bc)
        self.gamma = float(gamma)
        self.model = int(model)
        self.ncomp = self.ndim + 2 if model == EULER else 1
        inflow = dict(inflow or {})
        p = _Problem()
        p.model, p.ndim, p.gamma = self.model, self.ndim, self.gamma
        for d in range(3):
            p.n[d] = self.n[d] if d < self.ndim else 1
            p.h[d] = self.h[d] if d < self.ndim else 1.0
            for side in range(2):
                p.bc[d][side] = self.bc[d][side] if d < self.ndim else 0
        for d, (b0, b1) in enumerate(self.bc):
            if (b0 == BC_PERIODIC) != (b1 == BC_PERIODIC) or not all(0 <= b <= 3 for b in (b0, b1)):
                raise ValueError(f"bad boundary pair {self.bc[d]} in dimension {d}")
            for side, b in enumerate((b0, b1)):
                if b == BC_INFLOW:
                    prim = np.ascontiguousarray(inflow.pop((d, side)), dtype=np.float64)
                    if prim.shape != (self.ncomp,):
                        raise ValueError("inflow state needs ncomp primitive values")
                    q = np.zeros(5)
                    _load().or_inflow_conserved(ctypes.byref(p), _dp(prim), _dp(q))
                    for c in range(self.ncomp):
                        p.inflow[d][side][c] = q[c]
        if inflow:
            raise ValueError(f"inflow states given for sides that are not BC_INFLOW: {sorted(inflow)}")
        self._p = p

    def inflow_conserved(self, d: int, side: int) -> np.ndarray:
        """The conserved ghost state of an inflow side."""
        return np.array([self._p.inflow[d][side][c] for c in range(self.ncomp)])

    @property
    def shape(self):
        return (self.ncomp,) + self.n

    def centers(self, d: int) -> np.ndarray:
        """Cell centres x_i = lo + (i + 1/2) h along dimension d (0-based i)."""
        return self.lo[d] + (np.arange(self.n[d]) + 0.5) * self.h[d]

    def _check(self, U):
        if U.shape != self.shape or U.dtype != np.float64 or not U.flags.c_contiguous:
            raise ValueError(f"U must be C-contiguous float64 of shape {self.shape}")

    def alpha(self, U: np.ndarray) -> float:
        self._check(U)
        out = ctypes.c_double(0.0)
        s = _load().or_alpha(ctypes.byref(self._p), _dp(U), ctypes.byref(out))
        if s:
            raise OracleError(s)
        return out.value

    def interface_flux(self, U: np.ndarray, alpha: float, dim: int) -> np.ndarray:
        """F-hat along ``dim`` at the N_dim + 1 faces (face m between cells m-1 and m)."""
        self._check(U)
        shp = list(self.shape)
        shp[1 + dim] += 1
        F = np.zeros(shp)
        s = _load().or_interface_flux(ctypes.byref(self._p), float(alpha), _dp(U), int(dim), _dp(F))
        if s:
            raise OracleError(s)
        return F

    def rhs(self, U: np.ndarray, alpha: float, naive: bool = False) -> np.ndarray:
        self._check(U)
        L = np.zeros(self.shape)
        f = _load().or_rhs_naive if naive else _load().or_rhs
        s = f(ctypes.byref(self._p), float(alpha), _dp(U), _dp(L))
        if s:
            raise OracleError(s)
        return L

    def ssprk3(self, U: np.ndarray, dt: float, alphas=None):
        """One SSP-RK3 step in place. ``alphas``: the three stage alphas to use, or None to
        compute them exactly. Returns the alphas used."""
        self._check(U)
        al = np.zeros(3) if alphas is None else np.ascontiguousarray(alphas, dtype=np.float64).copy()
        s = _load().or_ssprk3(ctypes.byref(self._p), float(dt), 0 if alphas is None else 1, _dp(al), _dp(U))
        if s:
            raise OracleError(s)
        return al

    def run(self, U: np.ndarray, t_end: float, cfl: float = 0.5, fixed_dt: float = 0.0) -> int:
        self._check(U)
        n = ctypes.c_int64(0)
        s = _load().or_run(ctypes.byref(self._p), float(t_end), float(cfl), float(fixed_dt), _dp(U),
                           ctypes.byref(n))
        if s:
            raise OracleError(s)
        return n.value
