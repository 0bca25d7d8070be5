"""Thin Python face of the C ABI: one Simulation object per lbm_em handle.

PyTorch is only used for device memory and the stream handed to the
library (torch.cuda.current_stream() when a device is present); all lattice
Boltzmann arithmetic runs in liblbm_em.so.
"""
import ctypes as C
import json
import os

import numpy as np

from . import _lib as L

_POL = {"TM": L.TM, "TE": L.TE, "3D": L.D3}
_PREC = {"fp32": L.FP32, "fp64": L.FP64}


def _current_stream():
    try:
        import torch
    except ImportError:  # pragma: no cover - torch is part of the image
        return None
    if torch.cuda.is_available():
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return None


class Simulation:
    """One scattering instance on the GPU (see include/lbm_em.h)."""

    def __init__(self, nx, ny, nz=1, pol="TM", precision="fp32", absorb=(0, 0, 0), sigma_max=0.25,
                 stream=None):
        self.n = (int(nx), int(ny), int(nz))
        self.pol = pol
        self.precision = precision
        self.dtype = np.float32 if precision == "fp32" else np.float64
        cfg = L.Config()
        cfg.nx, cfg.ny, cfg.nz = self.n
        cfg.pol = _POL[pol]
        cfg.precision = _PREC[precision]
        for a in range(3):
            cfg.absorb[a] = int(absorb[a])
        cfg.sigma_max = float(sigma_max)
        cfg.stream = stream if stream is not None else _current_stream()
        h = C.c_void_p()
        L.check(L.lib().lbm_em_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self._theta_inc = 0.0
        self._has_mu = False      # permeability plane in use (a map or conductor cells)
        self._mu_user = False
        self._pec_set = False

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.check(L.lib().lbm_em_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inputs ----------------------------------------------------------
    def _set_material(self, fn, values, name):
        size = self.n[0] * self.n[1] * self.n[2]
        if hasattr(values, "data_ptr"):  # torch tensor
            t = values.contiguous()
            if t.numel() != size:
                raise ValueError(f"{name} has the wrong number of values")
            dt = {4: L.FP32, 8: L.FP64}[t.element_size()]
            where = L.DEVICE if t.is_cuda else L.HOST
            L.check(fn(self._h, C.c_void_p(t.data_ptr()), where, dt))
            return
        a = np.ascontiguousarray(values, dtype=np.float64)
        if a.size != size:
            raise ValueError(f"{name} has the wrong number of values")
        L.check(fn(self._h, a.ctypes.data_as(C.c_void_p), L.HOST, L.FP64))

    def set_permittivity(self, eps):
        """eps: numpy array or torch tensor with nx*ny*nz values ([z][y][x])."""
        self._set_material(L.lib().lbm_em_set_permittivity, eps, "eps")

    def set_permeability(self, mu):
        """mu_r(x) of a 2-D run, laid out like eps; None returns to mu_r = 1.
        Batches and the adjoint refuse a handle with a permeability map."""
        if mu is None:
            L.check(L.lib().lbm_em_set_permeability(self._h, None, L.HOST, L.FP64))
            self._mu_user = False
            self._has_mu = self._pec_set
            return
        self._set_material(L.lib().lbm_em_set_permeability, mu, "mu")
        self._mu_user = True
        self._has_mu = True

    def set_pec(self, mask):
        """Perfect-conductor cells of a TM run: boolean map laid out like eps
        (numpy, or a torch uint8/bool tensor); None removes the conductor."""
        if mask is None:
            L.check(L.lib().lbm_em_set_pec(self._h, None, L.HOST))
            self._pec_set = False
            self._has_mu = self._mu_user
            return
        size = self.n[0] * self.n[1] * self.n[2]
        if hasattr(mask, "data_ptr"):  # torch tensor
            import torch

            t = mask.contiguous().to(dtype=torch.uint8)
            if t.numel() != size:
                raise ValueError("mask has the wrong number of values")
            L.check(L.lib().lbm_em_set_pec(self._h, C.c_void_p(t.data_ptr()), L.DEVICE if t.is_cuda else L.HOST))
        else:
            a = np.ascontiguousarray(mask, dtype=np.uint8)
            if a.size != size:
                raise ValueError("mask has the wrong number of values")
            L.check(L.lib().lbm_em_set_pec(self._h, a.ctypes.data_as(C.c_void_p), L.HOST))
        self._pec_set = True
        self._has_mu = True

    def set_incident_line(self, enable=True):
        """Exact incident line for incidence along +-x or +-y (see
        lbm_em_set_incident_line): call after set_source, before stepping;
        farfield(incident=None) then uses the line instead of a companion."""
        L.check(L.lib().lbm_em_set_incident_line(self._h, 1 if enable else 0))

    def line_phasors(self):
        """The incident line's phasors, (n, 6) complex (Ex, Ey, Ez, Hx, Hy, Hz)."""
        n = C.c_int32()
        L.check(L.lib().lbm_em_get_line_phasors(self._h, None, C.byref(n)))
        out = np.zeros(n.value * 12)
        L.check(L.lib().lbm_em_get_line_phasors(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
        out = out.reshape(-1, 12)
        return out[:, 0::2] + 1j * out[:, 1::2]

    def set_source(self, lam, khat, ehat, amplitude=1.0, ramp_periods=3.0, center=None):
        pw = L.PlaneWave()
        pw.lam = float(lam)
        for a in range(3):
            pw.khat[a] = float(khat[a])
            pw.ehat[a] = float(ehat[a])
        pw.amplitude = float(amplitude)
        pw.ramp_periods = float(ramp_periods)
        c = center if center is not None else [(m - 1) / 2.0 for m in self.n]
        if self.n[2] == 1 and center is None:
            c = [c[0], c[1], 0.0]
        for a in range(3):
            pw.center[a] = float(c[a])
        L.check(L.lib().lbm_em_set_source(self._h, C.byref(pw)))
        self._khat = np.asarray(khat, float)
        self.lam = float(lam)

    def set_ntff(self, lo, hi, window_start, window_len):
        lo3 = (C.c_int32 * 3)(*(list(lo) + [0] * (3 - len(lo))))
        hi3 = (C.c_int32 * 3)(*(list(hi) + [0] * (3 - len(hi))))
        L.check(L.lib().lbm_em_set_ntff(self._h, lo3, hi3, int(window_start), int(window_len)))
        self.box = (tuple(lo), tuple(hi))

    # -- stepping ----------------------------------------------------------
    def step(self, n=1):
        L.check(L.lib().lbm_em_step(self._h, int(n)))

    def set_tile(self, vx, bx, by):
        L.check(L.lib().lbm_em_set_tile(self._h, int(vx), int(bx), int(by)))

    def set_fusion(self, steps_per_launch, tile=(0, 0)):
        """Time steps per launch (1 or 2) and the two-step tile (TX, TY);
        (0, 0) keeps the current tile."""
        L.check(L.lib().lbm_em_set_fusion(self._h, int(steps_per_launch), int(tile[0]), int(tile[1])))

    def get_fusion(self):
        v, tx, ty = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.lib().lbm_em_get_fusion(self._h, C.byref(v), C.byref(tx), C.byref(ty)))
        return v.value

    def get_fusion_tile(self):
        v, tx, ty = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.lib().lbm_em_get_fusion(self._h, C.byref(v), C.byref(tx), C.byref(ty)))
        return tx.value, ty.value

    def get_tile(self):
        v, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.lib().lbm_em_get_tile(self._h, C.byref(v), C.byref(b), C.byref(c)))
        return v.value, b.value, c.value

    def autotune(self, launches=20, cache=None):
        """Pick the fastest verified tile for this grid (see lbm_em_autotune).
        With a cache file (JSON; default $LBM_EM_TUNE_CACHE) a stored choice
        for the same arch / layout / precision / grid is reused."""
        cache = cache or os.environ.get("LBM_EM_TUNE_CACHE")
        key = _tune_key(self)
        table = {}
        if cache and os.path.exists(cache):
            table = json.load(open(cache))
            if key in table:
                self.set_tile(*table[key]["tile"])
                self.set_fusion(table[key]["fusion"], table[key]["fusion_tile"])
                return table[key]
        us = C.c_double()
        L.check(L.lib().lbm_em_autotune(self._h, int(launches), C.byref(us)))
        rec = {"tile": list(self.get_tile()), "fusion": self.get_fusion(),
               "fusion_tile": list(self.get_fusion_tile()), "us_per_step": us.value}
        if cache:
            table[key] = rec
            os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
            tmp = cache + ".tmp"
            json.dump(table, open(tmp, "w"), indent=1, sort_keys=True)
            os.replace(tmp, cache)
        return rec

    def reset(self):
        """Back to t = 0 with zero fields (inputs kept)."""
        L.check(L.lib().lbm_em_reset(self._h))

    @property
    def t(self):
        v = C.c_int64()
        L.check(L.lib().lbm_em_time(self._h, C.byref(v)))
        return v.value

    # -- outputs -----------------------------------------------------------
    def fields(self):
        """(E, H) at the current time as numpy arrays (nz, ny, nx, 3)."""
        shape = (self.n[2], self.n[1], self.n[0], 3)
        E = np.empty(shape, self.dtype)
        H = np.empty(shape, self.dtype)
        L.check(L.lib().lbm_em_get_fields(self._h, E.ctypes.data_as(C.c_void_p),
                                          H.ctypes.data_as(C.c_void_p), L.HOST))
        return E, H

    def fields_device(self):
        """(E, H) as torch CUDA tensors (nz, ny, nx, 3)."""
        import torch

        dt = torch.float32 if self.precision == "fp32" else torch.float64
        shape = (self.n[2], self.n[1], self.n[0], 3)
        E = torch.empty(shape, dtype=dt, device="cuda")
        H = torch.empty(shape, dtype=dt, device="cuda")
        L.check(L.lib().lbm_em_get_fields(self._h, C.c_void_p(E.data_ptr()), C.c_void_p(H.data_ptr()),
                                          L.DEVICE))
        return E, H

    def phasors(self):
        """Contour phasors: (X (p, 6) complex for the surface nodes in
        ascending linear index, probe (6,) complex)."""
        n = C.c_int32()
        L.check(L.lib().lbm_em_get_phasors(self._h, None, C.byref(n)))
        out = np.zeros((n.value + 1) * 12)
        L.check(L.lib().lbm_em_get_phasors(self._h, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
        out = out.reshape(-1, 12)
        X = out[:, 0::2] + 1j * out[:, 1::2]
        return X[:-1], X[-1]

    # -- inverse design ----------------------------------------------------
    def adjoint_setup(self, incident, theta_deg, dlo, dhi, weights=None, checkpoint_every=0):
        """Objective J = sum_a w_a |S(theta_a)|^2 against `incident`, design
        rectangle [dlo, dhi] (inclusive cell coordinates (x, y))."""
        th = np.ascontiguousarray(theta_deg, dtype=np.float64).ravel()
        w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64).ravel()
        lo = (C.c_int32 * 2)(*dlo)
        hi = (C.c_int32 * 2)(*dhi)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        L.check(L.lib().lbm_em_adjoint_setup(self._h, incident.handle, dp(th), dp(w) if w is not None else None,
                                             th.size, lo, hi, int(checkpoint_every)))
        self._design = (tuple(dlo), tuple(dhi))
        self._incident = incident

    def forward_checkpointed(self, n):
        J = C.c_double()
        L.check(L.lib().lbm_em_forward_checkpointed(self._h, int(n), C.byref(J)))
        # the handle keeps only the latest forward pass for lbm_em_backward
        self._forward_version = getattr(self, "_forward_version", 0) + 1
        return J.value

    def backward(self, device=False):
        """dJ/deps over the design rectangle, shape (ny_d, nx_d), float64."""
        (x0, y0), (x1, y1) = self._design
        shape = (y1 - y0 + 1, x1 - x0 + 1)
        if device:
            import torch

            g = torch.empty(shape, dtype=torch.float64, device="cuda")
            L.check(L.lib().lbm_em_backward(self._h, C.c_void_p(g.data_ptr()), L.DEVICE))
            return g
        g = np.empty(shape)
        L.check(L.lib().lbm_em_backward(self._h, g.ctypes.data_as(C.c_void_p), L.HOST))
        return g

    def farfield(self, theta_deg, phi_deg=None, incident=None):
        """|S|^2 at angles measured from the incidence direction (2-D: in
        the plane; 3-D: phi about khat from ehat).  incident: the companion
        run; None uses the incident line if one is set."""
        th = np.ascontiguousarray(theta_deg, dtype=np.float64).ravel()
        ph = None if phi_deg is None else np.ascontiguousarray(
            np.broadcast_to(phi_deg, th.shape), dtype=np.float64)
        out = np.empty(th.size)
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        L.check(L.lib().lbm_em_farfield(self._h, incident.handle if incident is not None else None,
                                        dp(th), dp(ph) if ph is not None else None, th.size, dp(out)))
        return out


def _tune_key(sim):
    try:
        import torch

        arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # pragma: no cover
        arch = "unknown"
    mu = "/mu" if sim._has_mu else ""
    return f"{arch}/{sim.pol}/{sim.precision}/{sim.n[0]}x{sim.n[1]}x{sim.n[2]}{mu}"


def step_many(sims, n):
    """Advance several 2-D Simulations together (one launch per step)."""
    arr = (C.c_void_p * len(sims))(*[s.handle.value for s in sims])
    L.check(L.lib().lbm_em_step_many(arr, len(sims), int(n)))


class Batch:
    """Reusable batch of 2-D Simulations stepped by one persistent launch
    per time step, replayed from captured HIP graphs."""

    def __init__(self, sims):
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s.handle.value for s in self.sims])
        b = C.c_void_p()
        L.check(L.lib().lbm_em_batch_create(arr, len(self.sims), C.byref(b)))
        self._b = b

    def step(self, n=1):
        L.check(L.lib().lbm_em_batch_step(self._b, int(n)))

    def set_grid(self, blocks):
        L.check(L.lib().lbm_em_batch_set_grid(self._b, int(blocks)))

    def autotune(self, launches=10):
        """Time every two-step tile on the batched instances (no state
        change) and keep the fastest; returns microseconds per step of all
        batched instances (see lbm_em_batch_autotune)."""
        us = C.c_double()
        L.check(L.lib().lbm_em_batch_autotune(self._b, int(launches), C.byref(us)))
        return us.value

    def set_cache_budget(self, nbytes):
        """Group instances so each group's state fits nbytes (0: one group)."""
        L.check(L.lib().lbm_em_batch_set_cache_budget(self._b, int(nbytes)))

    @property
    def groups(self):
        g = C.c_int32()
        L.check(L.lib().lbm_em_batch_groups(self._b, C.byref(g)))
        return g.value

    def tile(self):
        """(steps per launch, (TX, TY)) of the persistent kernel."""
        v, tx, ty = C.c_int32(), C.c_int32(), C.c_int32()
        L.check(L.lib().lbm_em_batch_get_tile(self._b, C.byref(v), C.byref(tx), C.byref(ty)))
        return v.value, (tx.value, ty.value)

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            L.check(L.lib().lbm_em_batch_destroy(self._b))
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def far_field_objective():
    """torch.autograd.Function computing J(eps_design) = sum_a w_a |S(theta_a)|^2
    for a Simulation prepared with adjoint_setup; the gradient comes from the
    library's discrete adjoint (lbm_em_backward)."""
    import torch

    class FarFieldIntensity(torch.autograd.Function):
        @staticmethod
        def forward(ctx, eps_design, sim, eps_full, steps):
            (x0, y0), (x1, y1) = sim._design
            full = eps_full.detach().clone().to(torch.float64)
            full.view(-1, full.shape[-2], full.shape[-1])[0, y0:y1 + 1, x0:x1 + 1] = eps_design.detach().to(
                torch.float64)
            sim.set_permittivity(full)
            J = sim.forward_checkpointed(steps)
            ctx.sim = sim
            ctx.version = sim._forward_version
            ctx.dev = eps_design.device
            ctx.dtype = eps_design.dtype
            return torch.tensor(J, dtype=torch.float64, device=eps_design.device)

        @staticmethod
        def backward(ctx, gJ):
            # the library holds the adjoint state of the handle's latest
            # forward pass only: a later forward (another J on the same
            # handle) would silently give that pass's gradient
            if getattr(ctx.sim, "_forward_version", None) != ctx.version:
                raise RuntimeError("FarFieldIntensity.backward: the simulation ran another forward pass after "
                                   "this one; its gradient is no longer available")
            g = ctx.sim.backward(device=ctx.dev.type == "cuda")
            g = torch.as_tensor(g, device=ctx.dev, dtype=torch.float64) * gJ
            return g.to(ctx.dtype), None, None, None

    return FarFieldIntensity
