"""The C ABI library loads and exports every function include/rmge.h declares.

CPU only: no call here reaches a device (argument validation and pure host
functions only).
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rmge.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(rmge_[A-Za-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def rmge():
    import paper_1406_5802_amd as m

    m.lib()
    return m


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("rmge_factor", "rmge_factor_ex", "rmge_solve", "rmge_solve_adjoint",
                 "rmge_factor_stats_get", "rmge_destroy", "rmge_status_string"):
        assert want in names


def test_library_exports_every_declared_symbol(rmge):
    lib = rmge.lib()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    from paper_1406_5802_amd import _rmge

    assert sorted(_rmge.EXPORTS) == _declared_functions()
    for name in _rmge.EXPORTS:
        assert callable(getattr(_rmge, name))


def test_host_only_entry_points(rmge):
    from paper_1406_5802_amd import _rmge

    assert _rmge.rmge_version() >= 100
    assert _rmge.rmge_param_count(1, 5) == 25
    assert _rmge.rmge_param_count(2, 5) == 5
    assert _rmge.rmge_param_count(3, 5) == 9
    assert _rmge.rmge_param_count(0, 5) == 0
    assert _rmge.rmge_param_count(1, 0) == 0
    assert "zero pivot" in _rmge.rmge_status_string(4)
    assert _rmge.rmge_status_string(99) == "unknown status"


def test_argument_validation_before_device(rmge):
    from paper_1406_5802_amd import _rmge

    fake = ctypes.c_void_p(0x1000).value  # never dereferenced: validation fails first
    assert _rmge.rmge_factor_ex(0, 8, 8, 1, 0, 64, 0, 0)[0] == _rmge.RMGE_EINVAL  # null A
    assert _rmge.rmge_factor_ex(fake, 8, 4, 1, 0, 64, 0, 0)[0] == _rmge.RMGE_EINVAL  # lda < n
    assert _rmge.rmge_factor_ex(fake, 8, 8, 7, 0, 64, 0, 0)[0] == _rmge.RMGE_EINVAL  # kind
    assert _rmge.rmge_factor_ex(fake, 8, 8, 1, 0, 300, 0, 0)[0] == _rmge.RMGE_EINVAL  # block
    assert _rmge.rmge_factor_ex(fake, 8, 8, 1, 0, 64, 5, 0)[0] == _rmge.RMGE_EINVAL  # prec
    assert _rmge.rmge_factor_ex(fake, 0, 8, 1, 0, 64, 0, 0)[0] == _rmge.RMGE_EINVAL  # n
    # Toeplitz FFT period above the LDS-resident maximum
    assert _rmge.rmge_factor_ex(fake, 9000, 9000, 3, 0, 64, 0, 0)[0] == _rmge.RMGE_EINVAL
    assert _rmge.rmge_solve(None, fake, 1, 1, fake, 1, 1, 0.0)[0] == _rmge.RMGE_EINVAL
    # row-exchange mode outside rmge_pivot
    assert _rmge.rmge_factor_pivoted(fake, 8, 8, 1, 0, 64, 0, 2, 0)[0] == _rmge.RMGE_EINVAL
    assert _rmge.rmge_factor_pivoted(fake, 8, 8, 1, 0, 64, 0, -1, 0)[0] == _rmge.RMGE_EINVAL
    assert _rmge.rmge_factors_perm(None, fake) == _rmge.RMGE_EINVAL
    assert _rmge.rmge_solve_gmres(None, 0, fake, 1, 1, fake, 1, 10, 8, 1e-14)[0] == _rmge.RMGE_EINVAL
    assert _rmge.rmge_solve_adjoint_ex(None, fake, 1, 1, fake, 1, 1, 0.0)[0] == _rmge.RMGE_EINVAL
    assert _rmge.rmge_factor_times(None)[0] == _rmge.RMGE_EINVAL


def test_binding_refuses_cpu_tensors(rmge):
    import torch

    with pytest.raises(TypeError):
        rmge.factor(torch.eye(4, dtype=torch.float64))


def test_package_is_not_the_oracle():
    # the product path never loads the oracle
    import sys

    import paper_1406_5802_amd  # noqa: F401

    src_dir = os.path.join(ROOT, "paper_1406_5802_amd")
    for fn in os.listdir(src_dir):
        if fn.endswith(".py"):
            text = open(os.path.join(src_dir, fn)).read()
            assert "import oracle" not in text and "from oracle" not in text, fn


def test_batch_create_rejects_bad_systems(rmge):
    # validated on the host before any device work
    from paper_1406_5802_amd import _rmge

    ok = _rmge.rmge_batch_system(10, _rmge.RMGE_MULT_GAUSSIAN, 1, 0, 0)
    for bad in (_rmge.rmge_batch_system(0, 1, 1, 0, 0), _rmge.rmge_batch_system(1025, 1, 1, 0, 0),
                _rmge.rmge_batch_system(10, _rmge.RMGE_MULT_TOEPLITZ, 1, 0, 0),
                _rmge.rmge_batch_system(10, 1, 1, -1, 0)):
        rc, _ = _rmge.rmge_batch_create([ok, bad], None, 16, 100)
        assert rc == _rmge.RMGE_EINVAL
    rc, _ = _rmge.rmge_batch_create([ok], None, 0, 100)  # restart out of range
    assert rc == _rmge.RMGE_EINVAL
    t = _rmge.rmge_batch_tuning((ctypes.c_int32 * 5)(16, 32, 48, 64, 64))
    rc, _ = _rmge.rmge_batch_create([ok], t, 16, 100)  # 48 is not a panel width
    assert rc == _rmge.RMGE_EINVAL
