"""The C-ABI library: it loads, exports every function include/mjk.h declares,
and rejects bad input on the host (no GPU needed for these)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2412_13203_amd import inputs, mjk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mjk.h")).read()
    return sorted(set(re.findall(r"\b(mjk_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_function():
    lib = mjk.lib()
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(mjk.EXPORTS)


def test_lmax():
    assert mjk.lib().mjk_lmax() >= 2


def test_nbf():
    cfg = inputs.make_config(2)
    assert mjk.nbf(cfg["basis"]) == 440


def _bad(basis, **changes):
    b = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in basis.items()}
    for k, (idx, val) in changes.items():
        b[k][idx] = val
    return b


@pytest.mark.parametrize("field,idx,val,code", [
    ("shell_l", 0, 5, -2),
    ("shell_l", 1, -1, -1),
    ("shell_nprim", 0, 7, -2),
    ("shell_nprim", 0, 0, -2),
    ("exps", 0, -1.0, -1),
    ("exps", 1, np.nan, -1),
    ("coefs", 2, np.inf, -1),
    ("shell_atom", 0, 99, -1),
    ("shell_prim_off", 3, 10 ** 6, -1),
])
def test_invalid_basis(field, idx, val, code):
    cfg = inputs.make_config(1)
    b = _bad(cfg["basis"], **{field: (idx, val)})
    with pytest.raises(mjk.MjkError) as ei:
        mjk.nbf(b)
    assert ei.value.code == code
    assert mjk.lib().mjk_last_error().decode()


def test_null_arguments():
    lib = mjk.lib()
    assert lib.mjk_nbf(None, None) == -1
    assert lib.mjk_ctx_create(0, None) == -1
    assert lib.mjk_build_jk(None, None, None, None, None) == -1
    assert lib.mjk_plan_bind(None, None, 0, None) == -1
    assert lib.mjk_schwarz(None, None) == -1


def test_no_device_error_is_clean():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    c = ctypes.c_void_p()
    rc = mjk.lib().mjk_ctx_create(0, ctypes.byref(c))
    assert rc == -3
    assert "device" in mjk.lib().mjk_last_error().decode()
