"""ctypes wrapper around the FP64 literal-scheme oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY -- used by tests/, the smoke check and the CPU
baseline of the benchmark; never by the product path.

The oracle runs the paper's scheme literally (section 2.1, Eq. LBGK_equation
and Eq. EDF): 42 doubles per cell, push streaming, open-boundary copy
(section 2.2), with the absorbing-layer / plane-wave readings documented in
lbm_oracle.c.  Arrays cross the boundary as C-contiguous float64 numpy
arrays indexed [z][y][x] (x fastest).
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        D = C.POINTER(C.c_double)
        I64 = C.c_int64
        L.oracle_create.restype = P
        L.oracle_create.argtypes = [C.c_int] * 6 + [C.c_double]
        L.oracle_destroy.argtypes = [P]
        L.oracle_set_eps.argtypes = [P, D]
        L.oracle_set_mu.argtypes = [P, D]
        L.oracle_set_pec.argtypes = [P, C.c_void_p]
        L.oracle_set_incident_line.restype = C.c_int
        L.oracle_set_incident_line.argtypes = [P, C.c_int]
        L.oracle_get_line_dft.argtypes = [P, D]
        L.oracle_set_source.argtypes = [P, C.c_double, D, D, C.c_double, C.c_double, D]
        L.oracle_clear_source.argtypes = [P]
        L.oracle_set_dft.argtypes = [P, I64, C.POINTER(I64), I64, I64]
        L.oracle_get_dft.argtypes = [P, D]
        L.oracle_time.restype = I64
        L.oracle_time.argtypes = [P]
        L.oracle_set_time.argtypes = [P, I64]
        L.oracle_get_state.argtypes = [P, D]
        L.oracle_set_state.argtypes = [P, D]
        L.oracle_fields.argtypes = [P, D, D]
        L.oracle_step.argtypes = [P, I64]
        L.oracle_threads.restype = C.c_int
        L.oracle_stream_transpose.argtypes = [P, D, D]
        L.oracle_stream_apply.argtypes = [P, D, D]
        L.oracle_adjoint.argtypes = [P, I64, I64, D, D, D]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def threads():
    """OpenMP threads the oracle runs with."""
    return lib().oracle_threads()


class Oracle:
    """FP64 literal D3Q7 electromagnetic LBM on an nx x ny x nz grid.

    absorb = (Wx, Wy, Wz): absorbing-layer width per axis, 0 for a periodic axis.
    """

    NV = 42

    def __init__(self, nx, ny, nz=1, absorb=(0, 0, 0), sigma_max=0.25):
        self.shape = (nz, ny, nx)
        self.n = (nx, ny, nz)
        self.absorb = tuple(int(w) for w in absorb)
        self.sigma_max = float(sigma_max)
        self._h = lib().oracle_create(nx, ny, nz, *self.absorb, self.sigma_max)
        if not self._h:
            raise ValueError("oracle_create rejected the grid / layer sizes")
        self.ncell = nx * ny * nz
        self._dft_n = 0
        self._line_n = 0

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    # -- media ---------------------------------------------------------
    def set_eps(self, eps):
        a = np.ascontiguousarray(np.broadcast_to(eps, self.shape), dtype=np.float64)
        lib().oracle_set_eps(self._h, _dp(a))

    def set_mu(self, mu):
        a = np.ascontiguousarray(np.broadcast_to(mu, self.shape), dtype=np.float64)
        lib().oracle_set_mu(self._h, _dp(a))

    def set_pec(self, mask):
        """Perfect-conductor cells (boolean map shaped like eps); None clears."""
        if mask is None:
            lib().oracle_set_pec(self._h, None)
            return
        self._pec = np.ascontiguousarray(np.broadcast_to(mask, self.shape), dtype=np.uint8)
        lib().oracle_set_pec(self._h, self._pec.ctypes.data_as(C.c_void_p))

    # -- plane wave ----------------------------------------------------
    def set_source(self, lam, khat, ehat, amp=1.0, ramp_periods=3.0, center=None):
        """Incident plane wave (reading): wavelength lam cells, direction khat,
        E polarisation ehat, ramp of ramp_periods periods (T = 3 lam steps)."""
        if center is None:
            center = [(n - 1) / 2.0 for n in self.n]
        kh = np.ascontiguousarray(khat, dtype=np.float64)
        eh = np.ascontiguousarray(ehat, dtype=np.float64)
        rc = np.ascontiguousarray(center, dtype=np.float64)
        self.lam = float(lam)
        lib().oracle_set_source(self._h, float(lam), _dp(kh), _dp(eh), float(amp),
                                float(ramp_periods) * 3.0 * float(lam), _dp(rc))

    def clear_source(self):
        lib().oracle_clear_source(self._h)

    def set_incident_line(self, axis):
        """Exact incident line along axis 0 (x), 1 (y) or 2 (z), None to remove it
        (lbm_oracle.c: the one-row auxiliary run and its layer rule).  Call
        after set_source and before stepping."""
        rc = lib().oracle_set_incident_line(self._h, -1 if axis is None else int(axis))
        if rc != 0:
            raise ValueError("the incident line needs a source along that axis")
        self._line_n = 0 if axis is None else self.n[int(axis)]

    def get_line_dft(self):
        """The line's phasors, shape (n_axis, 6): Ex, Ey, Ez, Hx, Hy, Hz."""
        out = np.zeros((max(self._line_n, 1), 12))
        lib().oracle_get_line_dft(self._h, _dp(out))
        out = out[: self._line_n]
        return out[:, 0::2] + 1j * out[:, 1::2]

    # -- DFT -----------------------------------------------------------
    def set_dft(self, cells, win0, winlen):
        """Fourier-transform E and H at the given linear cell indices over the
        steps [win0, win0 + winlen)."""
        c = np.ascontiguousarray(cells, dtype=np.int64)
        self._dft_n = c.size
        lib().oracle_set_dft(self._h, c.size, c.ctypes.data_as(C.POINTER(C.c_int64)),
                             int(win0), int(winlen))

    def get_dft(self):
        """Complex phasors, shape (ncells, 6): Ex, Ey, Ez, Hx, Hy, Hz."""
        out = np.zeros((max(self._dft_n, 1), 12))
        lib().oracle_get_dft(self._h, _dp(out))
        out = out[: self._dft_n]
        return out[:, 0::2] + 1j * out[:, 1::2]

    # -- state ---------------------------------------------------------
    @property
    def t(self):
        return lib().oracle_time(self._h)

    @t.setter
    def t(self, value):
        lib().oracle_set_time(self._h, int(value))

    def get_state(self):
        out = np.empty(self.shape + (7, 6))
        lib().oracle_get_state(self._h, _dp(out))
        return out

    def set_state(self, f):
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(self.shape + (7, 6))
        lib().oracle_set_state(self._h, _dp(a))

    def fields(self):
        """(E, H) of the current state, each shaped (nz, ny, nx, 3)."""
        E = np.empty(self.shape + (3,))
        H = np.empty(self.shape + (3,))
        lib().oracle_fields(self._h, _dp(E), _dp(H))
        return E, H

    def step(self, n=1):
        lib().oracle_step(self._h, int(n))

    # -- adjoint hooks ---------------------------------------------------
    def stream_apply(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.empty_like(x)
        lib().oracle_stream_apply(self._h, _dp(x), _dp(out))
        return out

    def stream_transpose(self, y):
        y = np.ascontiguousarray(y, dtype=np.float64)
        out = np.empty_like(y)
        lib().oracle_stream_transpose(self._h, _dp(y), _dp(out))
        return out

    def adjoint(self, history, dJdF, t0):
        """dJ/deps per cell from the stored forward states history[t]
        (pre-collision, t = t0 .. t0+T-1) and dJ/dF[t] (T, cells, 6)."""
        h = np.ascontiguousarray(history, dtype=np.float64)
        j = np.ascontiguousarray(dJdF, dtype=np.float64)
        T = h.shape[0]
        grad = np.empty(self.ncell)
        lib().oracle_adjoint(self._h, T, int(t0), _dp(h), _dp(j), _dp(grad))
        return grad.reshape(self.shape)
