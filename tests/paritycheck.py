"""Comparison helpers shared by the GPU parity tests (no method arithmetic).

Angular intensity bar (1e-3 relative on |S|^2), checked three ways:
  * nRMS      -- RMS of |S_gpu - S_oracle| over all angles / max S_oracle
                 (the paper's normalised RMS, section 3.2, Eq. rms_error);
  * max_abs   -- max over angles of |S_gpu - S_oracle| / max S_oracle, so a
                 miss at a single angle is not averaged away;
  * max_rel   -- max over angles of |S_gpu - S_oracle| / S_oracle(theta) at
                 every angle where S_oracle >= REL_FLOOR * max S_oracle.
The floor is explicit: the FP32 field error is relative to the field scale
of the whole grid, so near a deep minimum of |S|^2 (orders of magnitude
below the peak) the error relative to the local value is not a meaningful
bar; there the absolute check (max_abs) applies.
"""
import sys

import numpy as np

REL_FLOOR = 1e-2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def intensity_errors(S_g, S_o, floor=REL_FLOOR):
    S_g = np.asarray(S_g, dtype=np.float64)
    S_o = np.asarray(S_o, dtype=np.float64)
    assert S_g.shape == S_o.shape and np.all(np.isfinite(S_g))
    m = S_o.max()
    d = np.abs(S_g - S_o)
    mask = S_o >= floor * m
    return {"nrms": float(np.sqrt(np.mean(d ** 2)) / m), "max_abs": float(d.max() / m),
            "max_rel": float((d[mask] / S_o[mask]).max()), "rel_angles": int(mask.sum())}


def assert_intensity(S_g, S_o, tol, tag="", floor=REL_FLOOR):
    e = intensity_errors(S_g, S_o, floor)
    say(tag, "|S|^2 errors", e)
    assert e["nrms"] <= tol, (tag, e)
    assert e["max_abs"] <= tol, (tag, e)
    assert e["max_rel"] <= tol, (tag, e)
    return e


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def max_rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())
