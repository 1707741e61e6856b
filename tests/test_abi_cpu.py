"""The C ABI on a machine without a GPU: the library loads, exports every
entry point include/purse.h declares, and host-side validation returns the
documented error codes without launching anything."""
import ctypes
import os
import re

import pytest

from paper_2403_09990_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "purse.h")).read()
    return set(re.findall(r"^(?:purse_status|const char \*)\s*(purse_\w+)\(", text, re.M))


def test_header_declares_what_the_binding_wraps():
    assert _declared() == set(_native.EXPORTED)


def test_header_constants_match_the_binding():
    """Every PURSE_* integer constant of the header has the same value in the
    Python binding."""
    text = open(os.path.join(ROOT, "include", "purse.h")).read()
    defs = dict(re.findall(r"^#define\s+(PURSE_\w+)\s+(\(?-?\d+(?:\s*<<\s*\d+)?\)?)", text, re.M))
    enums = dict(re.findall(r"^\s+(PURSE_\w+)\s*=\s*(-?\d+)", text, re.M))
    defs.update(enums)
    assert len(defs) >= 20
    for name, expr in defs.items():
        if name.startswith("PURSE_MAX_KP") or not hasattr(_native, name):
            continue
        assert getattr(_native, name) == eval(expr), name
    for name in dir(_native):
        if name.startswith("PURSE_") and not name.startswith("PURSE_MAX"):
            assert name in defs, name


def test_library_exports_every_declared_symbol():
    lib = _native.load()
    for name in _declared():
        assert hasattr(lib, name), name


def _batch(fake=0x10000):
    b = _native.PurseBatch(n_inst=1, max_kp=8, total_kp=8, total_samples=1024, max_samples=1024)
    for f in ("kind", "n_kp", "kp_off", "sample_off", "model_pts", "centres", "shapes", "bounds",
              "intrinsics", "seed"):
        setattr(b, f, fake)
    return b


def _params():
    p = _native.PurseParams()
    assert _native.load().purse_default_params(ctypes.byref(p)) == _native.PURSE_OK
    return p


def test_default_params():
    p = _params()
    assert (p.n_iters, p.n_gn, p.n_bis, p.megb_iters, p.megb_avg) == (50, 2, 16, 4096, 10)
    assert abs(p.kappa - 0.999) < 1e-7 and abs(p.omega0 - 0.5) < 1e-7 and abs(p.v0 - 0.2) < 1e-7
    assert _native.load().purse_default_params(None) == _native.PURSE_E_NULL


def test_workspace_size_grows_with_samples():
    lib = _native.load()
    p = _params()
    n1, n2 = ctypes.c_size_t(), ctypes.c_size_t()
    b = _batch()
    assert lib.purse_workspace_size(ctypes.byref(b), ctypes.byref(p), ctypes.byref(n1)) == 0
    b.total_samples = b.max_samples = 4096
    assert lib.purse_workspace_size(ctypes.byref(b), ctypes.byref(p), ctypes.byref(n2)) == 0
    assert n2.value > n1.value > 0 and n1.value % 256 == 0


@pytest.mark.parametrize("field,value,code", [
    ("n_inst", 0, _native.PURSE_E_BAD_ARG),
    ("max_kp", 2, _native.PURSE_E_BAD_ARG),
    ("max_kp", 65, _native.PURSE_E_BAD_ARG),
    ("total_samples", 0, _native.PURSE_E_BAD_ARG),
    ("max_samples", 2048, _native.PURSE_E_BAD_ARG),
    ("kind", None, _native.PURSE_E_NULL),
    ("seed", None, _native.PURSE_E_NULL),
])
def test_batch_validation(field, value, code):
    lib = _native.load()
    b = _batch()
    setattr(b, field, value)
    n = ctypes.c_size_t()
    assert lib.purse_workspace_size(ctypes.byref(b), ctypes.byref(_params()), ctypes.byref(n)) == code
    assert lib.purse_last_error().decode() != ""


@pytest.mark.parametrize("field,value", [
    ("n_iters", -1), ("n_gn", 0), ("n_bis", 31), ("megb_iters", 0), ("megb_avg", 5000),
    ("kappa", 0.0), ("kappa", 1.5), ("tau_abs_3d", -1.0), ("z_min", 0.0), ("tile", 100),
    ("ckpt_every", 0), ("omega0", -0.1)])
def test_param_validation(field, value):
    lib = _native.load()
    p = _params()
    setattr(p, field, value)
    n = ctypes.c_size_t()
    assert lib.purse_workspace_size(ctypes.byref(_batch()), ctypes.byref(p), ctypes.byref(n)) \
        == _native.PURSE_E_BAD_ARG


def test_sample_argument_errors_without_device():
    lib = _native.load()
    b, p = _batch(), _params()
    n = ctypes.c_size_t()
    assert lib.purse_workspace_size(ctypes.byref(b), ctypes.byref(p), ctypes.byref(n)) == 0
    fake = 0x100000
    # NULL outputs
    assert lib.purse_sample(ctypes.byref(b), ctypes.byref(p), None, fake, fake, fake, n.value, None) \
        == _native.PURSE_E_NULL
    # misaligned / small workspace
    assert lib.purse_sample(ctypes.byref(b), ctypes.byref(p), fake, fake, fake, fake + 4, n.value, None) \
        == _native.PURSE_E_WORKSPACE
    assert lib.purse_sample(ctypes.byref(b), ctypes.byref(p), fake, fake, fake, fake, n.value - 1, None) \
        == _native.PURSE_E_WORKSPACE
    import torch
    if not torch.cuda.is_available():
        # every argument valid: the call reaches the device check and stops there
        assert lib.purse_sample(ctypes.byref(b), ctypes.byref(p), fake, fake, fake, fake, n.value, None) \
            == _native.PURSE_E_NO_DEVICE
        assert lib.purse_megb(ctypes.byref(b), ctypes.byref(p), fake, fake, fake, fake, fake, fake, fake,
                              fake, n.value, None) == _native.PURSE_E_NO_DEVICE


def test_status_strings():
    lib = _native.load()
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert lib.purse_status_string(code)


def test_sample_noalloc_limits_without_device():
    """The allocation-free sampler rejects batches beyond its static scratch
    on the host, before any device call."""
    lib = _native.load()
    p = _params()
    fake = 0x100000
    b = _batch()
    b.n_inst, b.total_kp = 1025, 1025 * 8
    assert lib.purse_sample_noalloc(ctypes.byref(b), ctypes.byref(p), fake, fake, fake, None) \
        == _native.PURSE_E_BAD_ARG
    b = _batch()
    b.n_inst, b.max_kp, b.total_kp = 1024, 64, 65537
    assert lib.purse_sample_noalloc(ctypes.byref(b), ctypes.byref(p), fake, fake, fake, None) \
        == _native.PURSE_E_BAD_ARG
    b = _batch()
    assert lib.purse_sample_noalloc(ctypes.byref(b), ctypes.byref(p), None, fake, fake, None) \
        == _native.PURSE_E_NULL
    import torch
    if not torch.cuda.is_available():
        assert lib.purse_sample_noalloc(ctypes.byref(b), ctypes.byref(p), fake, fake, fake, None) \
            == _native.PURSE_E_NO_DEVICE
