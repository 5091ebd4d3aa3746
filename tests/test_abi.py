"""The C ABI library loads and exports every function that include/qo.h declares
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "qo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qo_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_2605_25149_amd import binding

    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_all_symbols():
    from paper_2605_25149_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libqo_hip.so not built")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_without_gpu():
    from paper_2605_25149_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libqo_hip.so not built")
    lib = binding.load_library()
    assert lib.qo_status_string(0) == b"QO_OK"
    assert lib.qo_status_string(6) == b"QO_ERR_PCG_NOCONV"


def test_create_rejects_bad_config_before_device_work():
    """Argument validation happens before any HIP call (so it runs without a GPU)."""
    from paper_2605_25149_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libqo_hip.so not built")
    lib = binding.load_library()
    cfg = binding.QoConfig()
    cfg.dim = 4
    h = ctypes.c_void_p()
    assert lib.qo_create(ctypes.byref(cfg), None, ctypes.byref(h)) == binding.QO_ERR_ARG
    cfg.dim = 2
    cfg.n[0], cfg.n[1] = 8, 8
    cfg.L[0] = cfg.L[1] = 1.0
    cfg.kinetic = 0.5
    cfg.N = 64  # N >= Ng
    cfg.pcg_tol, cfg.pcg_maxit, cfg.pcg_check = 1e-10, 100, 4
    assert lib.qo_create(ctypes.byref(cfg), None, ctypes.byref(h)) == binding.QO_ERR_ARG
    cfg.N = 4
    cfg.precision = 1
    cfg.refine_inner_tol = 0.0
    assert lib.qo_create(ctypes.byref(cfg), None, ctypes.byref(h)) == binding.QO_ERR_ARG
    assert lib.qo_create(None, None, ctypes.byref(h)) == binding.QO_ERR_ARG
