"""Host-side checks of the C ABI that need no GPU.

* libvemb.so loads and exports every function declared in include/vemb.h;
* argument validation happens before any device work, so invalid problem
  specifications return their error codes on a machine without a GPU.
"""
import ctypes
import os
import re

import pytest

from paper_2106_02682_amd import vemb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "vemb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vemb_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = vemb.lib()
    names = _declared_functions()
    assert len(names) >= 13
    for name in names:
        assert hasattr(lib, name), name
    assert set(vemb.EXPORTS) <= set(names)


def _err(fn):
    with pytest.raises(vemb.VembError) as ei:
        fn()
    return ei.value.code


TFI = [(-1.0, (("X", (0, 0)),)), (-1.0, (("Z", (0, 0)), ("Z", (1, 0))))]


def test_invalid_specs_are_rejected_before_device_work():
    null = vemb.ctypes.c_void_p(None)
    assert _err(lambda: vemb.create_problem(TFI, (8, 1), (3, 1), stream=null)) == -1  # does not tile
    assert _err(lambda: vemb.create_problem(TFI, (4, 1), (4, 1), stream=null)) == -2  # one cluster
    assert _err(lambda: vemb.create_problem(TFI, (10, 1), (5, 1), stream=null)) == -2  # L > 4
    assert _err(lambda: vemb.create_problem(TFI, (8, 1), (1, 1), mu=-1.0, stream=null)) == -1
    three = [(1.0, (("Z", (0, 0)), ("Z", (1, 0)), ("Z", (2, 0))))]
    assert _err(lambda: vemb.create_problem(three, (8, 1), (1, 1), stream=null)) == -2
    assert _err(lambda: vemb.create_problem([(1.0, (("Y", (0, 0)),))], (4, 1), (1, 1), stream=null)) == -2
    # last_error carries a message
    assert b"" != vemb.lib().vemb_last_error()


def test_null_arguments():
    lib = vemb.lib()
    assert lib.vemb_create_problem(None, None, None, None, None, None) == -1
    assert lib.vemb_step(None, 1) == -1
    assert lib.vemb_dual_bound(None, None) == -1
    assert lib.vemb_psd_project_batched(None, None, 4, 1, 0, 0, None) == -1
    lib.vemb_destroy(None)  # no-op
    assert lib.vemb_batch_create(None, 0, 1, None) == -1
    arr = (ctypes.c_void_p * 2)(None, None)
    out = ctypes.c_void_p()
    assert lib.vemb_batch_create(arr, 2, 1, ctypes.byref(out)) == -1
    assert lib.vemb_batch_step(None, 1) == -1
    assert lib.vemb_batch_dual_bounds(None, None, None) == -1
    lib.vemb_batch_destroy(None)  # no-op


def test_dense_specs_are_rejected_before_device_work():
    null = vemb.ctypes.c_void_p(None)
    assert _err(lambda: vemb.Dense(TFI, (8, 1), (3, 1), stream=null)) == -1  # does not tile
    assert _err(lambda: vemb.Dense(TFI, (4, 1), (4, 1), stream=null)) == -2  # one cluster
    # K = M n_op = 10 * 256 above the largest dense projection (1024)
    assert _err(lambda: vemb.Dense(TFI, (40, 1), (4, 1), stream=null)) == -2
    # fields: Y is not real, coefficients must be finite
    assert _err(lambda: vemb.Dense(TFI, (8, 1), (2, 1), fields=[("Y", (0, 0), 1.0)], stream=null)) == -2
    assert _err(lambda: vemb.Dense(TFI, (8, 1), (2, 1), fields=[("X", (0, 0), float("nan"))], stream=null)) == -1
    lib = vemb.lib()
    assert lib.vemb_dense_create(None, None, None, None, 0, None, None, None) == -1
    assert lib.vemb_dense_step(None, 1) == -1
    assert lib.vemb_dense_dual_bound(None, None) == -1
    assert lib.vemb_dense_primal_energy(None, None, None) == -1
    assert lib.vemb_dense_get_state(None, None) == -1
    assert lib.vemb_dense_set_state(None, None) == -1
    assert lib.vemb_dense_last_sweeps(None, None, None) == -1
    lib.vemb_dense_destroy(None)  # no-op


def test_fermionic_specs_are_rejected_before_device_work():
    null = vemb.ctypes.c_void_p(None)
    hop = [(-1.0, (("F", (0, 0)), ("F", (1, 0))))]
    # hopping terms need a fermionic problem; fermionic problems need the complete collection
    assert _err(lambda: vemb.create_problem(hop, (8, 1), (2, 1), stream=null)) == -1
    assert _err(lambda: vemb.create_problem(hop, (8, 1), (2, 1), opset="pauli1", fermionic=True, stream=null)) == -2
    # X / Y letters have no fermionic meaning here; a lone hopping end is malformed
    assert _err(lambda: vemb.create_problem(hop + TFI[:1], (8, 1), (2, 1), fermionic=True, stream=null)) == -2
    assert _err(lambda: vemb.create_problem([(1.0, (("F", (0, 0)),))], (8, 1), (2, 1), fermionic=True,
                                            stream=null)) == -1
    # dense: fermionic fields are Z only
    assert _err(lambda: vemb.Dense(hop, (8, 1), (2, 1), fields=[("X", (0, 0), 0.3)], fermionic=True,
                                   stream=null)) == -2


def test_sign_projection_rejects_bad_sizes():
    lib = vemb.lib()
    assert lib.vemb_psd_project_sign(None, None, 16, None) == -1
    buf = ctypes.c_void_p(1)
    assert lib.vemb_psd_project_sign(buf, buf, 24, None) == -1
    assert lib.vemb_psd_project_sign(buf, buf, 0, None) == -1
    assert lib.vemb_psd_project_sign(buf, buf, 8192, None) == -1
