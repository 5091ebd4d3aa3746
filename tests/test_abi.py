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


def test_binding_structs_match_header():
    """The ctypes mirrors of qo_config / qo_step_stats list the header's members in order."""
    from paper_2605_25149_amd import binding

    src = open(os.path.join(ROOT, "include", "qo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    for cname, py in [("qo_config", binding.QoConfig), ("qo_step_stats", binding.QoStepStats)]:
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", src).group(1)
        names = []
        for decl in body.split(";"):
            toks = decl.strip().split(None, 1)
            if len(toks) == 2:
                names += [re.sub(r"\[.*\]", "", v.strip()) for v in toks[1].split(",")]
        assert names == [f[0] for f in py._fields_], cname


def test_create_rejects_bad_precond_before_device_work():
    """The fast-Poisson preconditioner's limits are checked before any HIP call."""
    from paper_2605_25149_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libqo_hip.so not built")
    lib = binding.load_library()
    cfg = binding.QoConfig()
    cfg.dim = 3
    cfg.n[0], cfg.n[1], cfg.n[2] = 257, 200, 200  # an axis of more than 256 points
    for k in range(3):
        cfg.L[k] = 1.0
    cfg.kinetic, cfg.N = 0.5, 4
    cfg.pcg_tol, cfg.pcg_maxit, cfg.pcg_check = 1e-10, 100, 4
    cfg.precond = 1
    h = ctypes.c_void_p()
    assert lib.qo_create(ctypes.byref(cfg), None, ctypes.byref(h)) == binding.QO_ERR_ARG
    cfg.n[0] = cfg.n[1] = cfg.n[2] = 32
    cfg.pcg_variant = 1  # the one-sweep form has no preconditioner hook
    assert lib.qo_create(ctypes.byref(cfg), None, ctypes.byref(h)) == binding.QO_ERR_ARG
    cfg.pcg_variant = 0
    cfg.precond = 2
    assert lib.qo_create(ctypes.byref(cfg), None, ctypes.byref(h)) == binding.QO_ERR_ARG


def test_noalloc_gram_validates_before_device_work():
    """qo_gram_pair_noalloc checks its arguments before any HIP call: null pointers, ld < ng
    and ncols beyond QO_NOALLOC_MAX_COLS give QO_ERR_ARG and a message from
    qo_last_error(NULL) (runs without a GPU)."""
    from paper_2605_25149_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("libqo_hip.so not built")
    lib = binding.load_library()
    fake = ctypes.c_void_p(4096)  # never dereferenced: every call below fails validation
    f = lib.qo_gram_pair_noalloc
    assert f(None, fake, 100, 100, 4, 1.0, fake, None) == binding.QO_ERR_ARG
    assert b"null pointer" in lib.qo_last_error(None)
    assert f(fake, fake, 99, 100, 4, 1.0, fake, None) == binding.QO_ERR_ARG
    assert f(fake, fake, 100, 100, 1025, 1.0, fake, None) == binding.QO_ERR_ARG
    assert b"ncols 1025" in lib.qo_last_error(None)
    assert f(fake, fake, 100, 100, 0, 1.0, fake, None) == binding.QO_ERR_ARG
    assert f(fake, fake, 100, 100, 4, 0.0, fake, None) == binding.QO_ERR_ARG
