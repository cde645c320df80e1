"""The C-ABI library loads, exports every function include/dfjk.h declares,
and rejects bad arguments before touching a device.  Runs without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dfjk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfjk_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2506_06661_amd as pkg
    return pkg.lib()


def test_exports_every_declared_function(L):
    names = declared_functions()
    assert "dfjk_init" in names and "dfjk_build_J" in names and "dfjk_build_K" in names
    for n in names:
        assert hasattr(L, n), n


def test_invalid_arguments(L):
    import paper_2506_06661_amd as pkg
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(4096)
    assert L.dfjk_init(None, fake, 0, 4, 4, 10, None, None) == -1
    assert L.dfjk_init(ctypes.byref(h), None, 0, 4, 4, 10, None, None) == -1
    assert "null B" in pkg.dfjk_last_error()
    assert L.dfjk_init(ctypes.byref(h), fake, 9, 4, 4, 10, None, None) == -1
    assert L.dfjk_init(ctypes.byref(h), fake, 0, 0, 4, 10, None, None) == -1
    assert L.dfjk_init(ctypes.byref(h), fake, 0, 4, 0, 10, None, None) == -1
    assert L.dfjk_init(ctypes.byref(h), fake, 0, 4, 4, 9, None, None) == -1  # ldB < npair
    assert "ldB" in pkg.dfjk_last_error()
    assert L.dfjk_build_J(None, fake, fake, None) == -1
    assert L.dfjk_build_J_diag(None, fake, fake, None, fake) == -1
    assert L.dfjk_build_J_multi(None, 2, fake, fake, None) == -1
    assert L.dfjk_form_B(0, 5, fake, fake, 5, None) == -1
    assert L.dfjk_form_B(4, 5, fake, fake, 4, None) == -1  # ldQ < ncol
    assert L.dfjk_build_K(None, fake, 3, None, fake) == -1
    assert L.dfjk_build_K_factored(None, fake, 3, None, ctypes.c_double(1.0), fake) == -1
    assert L.dfjk_build_K_pair(None, fake, fake, 3, 0, ctypes.c_double(1.0), fake) == -1
    g = ctypes.c_double()
    L.dfjk_probe_hbm_read.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_double)]
    assert L.dfjk_probe_hbm_read(None, 1024, ctypes.byref(g)) == -1
    assert L.dfjk_probe_hbm_read(ctypes.c_void_p(4097), 1024, ctypes.byref(g)) == -1  # not 16-byte aligned
    n = ctypes.c_size_t()
    assert L.dfjk_workspace_bytes(None, ctypes.byref(n)) == -1
    L.dfjk_destroy(None)  # no-op
    assert L.dfjk_quantize(None, fake, 2, 10, None) == -1
    assert L.dfjk_quantize(fake, fake, 0, 10, None) == -1  # F64 is not a reduced format


def test_no_device_reported():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_2506_06661_amd as pkg
    L = pkg.lib()
    h = ctypes.c_void_p()
    assert L.dfjk_init(ctypes.byref(h), ctypes.c_void_p(4096), 0, 4, 4, 10, None, None) == -2
    assert "no HIP device" in pkg.dfjk_last_error()


def test_batch_invalid_arguments(L):
    import paper_2506_06661_amd as pkg
    from paper_2506_06661_amd.dfjk import Mol
    b = ctypes.c_void_p()
    arr = (Mol * 1)()
    arr[0] = Mol(4096, 4, 8, 10, 2, 4096, 4096, 4096, 4096)
    assert L.dfjk_batch_init(None, arr, 1, 1, None) == -1
    assert L.dfjk_batch_init(ctypes.byref(b), arr, 0, 1, None) == -1
    assert L.dfjk_batch_init(ctypes.byref(b), arr, 1, 0, None) == -5  # FP64 is not batched
    arr[0] = Mol(4096, 4, 8, 9, 2, 4096, 4096, 4096, 4096)              # ldB < npair
    assert L.dfjk_batch_init(ctypes.byref(b), arr, 1, 1, None) == -1
    assert "molecule 0" in pkg.dfjk_last_error()
    assert L.dfjk_batch_build(None) == -1
    assert L.dfjk_batch_launch(None) == -1
    assert L.dfjk_batch_set_k16(None, 1) == -1
    L.dfjk_batch_destroy(None)


def test_scf_invalid_arguments(L):
    fake = ctypes.c_void_p(4096)
    assert L.dfjk_scf_step(None, fake, fake, fake, 2, 0, None) == -1
    assert L.dfjk_scf_reset(None) == -1


def test_reserved_options_invalid(L):
    import paper_2506_06661_amd as pkg
    fake = ctypes.c_void_p(4096)
    assert L.dfjk_update_B(None) == -1
    # option ranges are checked before the device is touched
    o = pkg.dfjk.default_options()
    assert o.max_ncol == 0 and o.max_ndm == 8
    o.max_ncol = 5  # > nao = 4
    h = ctypes.c_void_p()
    assert L.dfjk_init(ctypes.byref(h), fake, 0, 4, 4, 10, None, ctypes.byref(o)) == -1
    assert "max_ncol" in pkg.dfjk_last_error()
    o.max_ncol, o.max_ndm = 2, 0
    assert L.dfjk_init(ctypes.byref(h), fake, 0, 4, 4, 10, None, ctypes.byref(o)) == -1


def test_static_invalid_arguments(L):
    import paper_2506_06661_amd as pkg
    fake = ctypes.c_void_p(4096)
    # dfjk_build_J_static checks its arguments before any device call
    assert L.dfjk_build_J_static(None, 0, 4, 4, 10, None, None, fake, fake, None) == -1
    assert L.dfjk_build_J_static(fake, 9, 4, 4, 10, None, None, fake, fake, None) == -1
    assert L.dfjk_build_J_static(fake, 0, 4, 4, 9, None, None, fake, fake, None) == -1  # ldB < npair
    assert "ldB" in pkg.dfjk_last_error()
    assert L.dfjk_build_J_static(fake, 0, 4, 4, 10, None, None, None, fake, None) == -1
    o = pkg.dfjk.default_options()
    o.compensated_j = 7
    assert L.dfjk_build_J_static(fake, 1, 4, 4, 10, None, ctypes.byref(o), fake, fake, None) == -1
    assert L.dfjk_static_scratch_bytes() == 128 << 20
