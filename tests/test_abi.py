"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, and reports a missing device as an error code (no abort)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm_em.h")).read()
    return sorted(set(re.findall(r"\b(lbm_em_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_2510_11042_amd import _lib

    assert sorted(_lib.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2510_11042_amd import _lib

    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_errors_are_status_codes_without_device():
    import torch

    if torch.cuda.is_available():
        pytest.skip("device present: covered by the GPU tests")
    from paper_2510_11042_amd import _lib

    L = _lib.lib()
    cfg = _lib.Config()
    cfg.nx, cfg.ny, cfg.nz, cfg.pol, cfg.precision = 16, 16, 1, 0, 0
    h = C.c_void_p()
    st = L.lbm_em_create(C.byref(cfg), C.byref(h))
    assert st == _lib.EDEVICE
    assert b"device" in L.lbm_em_last_error()
    cfg.nx = 0
    assert L.lbm_em_create(C.byref(cfg), C.byref(h)) == _lib.EINVAL
    cfg.nx, cfg.absorb[0] = 16, 9            # 2W > n
    assert L.lbm_em_create(C.byref(cfg), C.byref(h)) == _lib.EINVAL
    assert L.lbm_em_create(None, C.byref(h)) == _lib.EINVAL
    assert L.lbm_em_step(None, 1) == _lib.EINVAL
    # one population plane (rows padded to 64 cells) must stay below 4 GiB
    cfg.absorb[0] = 0
    cfg.nx, cfg.ny = 32768, 32768                      # FP32: exactly 4 GiB
    assert L.lbm_em_create(C.byref(cfg), C.byref(h)) == _lib.EINVAL
    assert b"4 GiB" in L.lbm_em_last_error()
    cfg.nx = 32705                                     # padded to 32768: still 4 GiB
    assert L.lbm_em_create(C.byref(cfg), C.byref(h)) == _lib.EINVAL
    cfg.nx, cfg.ny = 32768, 32767                      # just below: passes to the device query
    assert L.lbm_em_create(C.byref(cfg), C.byref(h)) == _lib.EDEVICE
    cfg.precision, cfg.nx, cfg.ny = 1, 16384, 32768    # FP64: exactly 4 GiB
    assert L.lbm_em_create(C.byref(cfg), C.byref(h)) == _lib.EINVAL
