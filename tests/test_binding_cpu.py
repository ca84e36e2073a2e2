"""CPU checks of the Python binding's argument validation: every entry point
that hands tensors to the library rejects a mismatched dtype, shape,
contiguity or device with a ValueError before any library call (the kernels
take element sizes and extents from the vectors, so a complex64 eps_c next
to complex128 vectors would be read out of bounds)."""
import numpy as np
import pytest
import torch

from paper_1811_00484_amd import vie


class _FakeOp:
    """Stands in for an operator: the checks read only its grid."""

    def __init__(self, n):
        self.n = n
        self.handle = None


N = (5, 4, 3)
SHAPE = (3, 3, 4, 5)
GRID = (3, 4, 5)


def _v(dtype=torch.complex128, shape=SHAPE):
    return torch.zeros(shape, dtype=dtype)


def _raises(fn, *a, **k):
    with pytest.raises(ValueError) as ei:
        fn(*a, **k)
    return str(ei.value)


def test_matvec_rejects_mismatched_eps_c_and_out():
    op = _FakeOp(N)
    x = _v()
    assert "dtype" in _raises(vie.matvec, op, x, _v(torch.complex64, GRID))
    assert "shape" in _raises(vie.matvec, op, x, _v(shape=(3, 4, 4)))
    assert "contiguous" in _raises(vie.matvec, op, x, _v(shape=(5, 4, 3)).permute(2, 1, 0))
    assert "required" in _raises(vie.matvec, op, x, None)
    assert "dtype" in _raises(vie.matvec, op, x, _v(shape=GRID), out=_v(torch.complex64))
    # consistent host tensors: refused as host memory
    assert "device tensor" in _raises(vie.matvec, op, x, _v(shape=GRID))
    assert "device tensor" in _raises(vie.matvec, op, x, kind="N")


def test_solve_rejects_mismatched_eps_c_and_x0():
    op = _FakeOp(N)
    b = _v()
    assert "dtype" in _raises(vie.solve, op, b, _v(torch.complex64, GRID))
    assert "required" in _raises(vie.solve, op, b, None)
    assert "dtype" in _raises(vie.solve, op, b, _v(shape=GRID), x0=_v(torch.complex64))
    assert "shape" in _raises(vie.solve, op, b, _v(shape=GRID), x0=_v(shape=(2,) + SHAPE))
    assert "device tensor" in _raises(vie.solve, op, b, _v(shape=GRID), x0=_v())


def test_multi_instance_calls_reject_mismatches():
    op = _FakeOp(N)
    b = _v().unsqueeze(0)
    good = _v(shape=GRID)
    bad = _v(torch.complex64, GRID)
    assert "dtype" in _raises(vie.matvec_multi, [(op, b, good), (op, b, bad)])
    assert "required" in _raises(vie.matvec_multi, [(op, b, None)])
    assert "dtype" in _raises(vie.solve_multi, [(op, b, bad)])
    assert "required" in _raises(vie.solve_multi, [(op, b, None)])
    assert "one tensor per instance" in _raises(vie.solve_multi, [(op, b, good)], x0=[])
    assert "dtype" in _raises(vie.solve_multi, [(op, b, good)], x0=[_v(torch.complex64).unsqueeze(0)])
    assert "share a dtype" in _raises(vie.solve_multi, [(op, b, good), (op, b.to(torch.complex64), bad)])
    assert "device tensor" in _raises(vie.solve_multi, [(op, b, good)])


def test_field_helpers_reject_mismatches():
    op = _FakeOp(N)
    e_inc = _v(shape=(3,) + GRID)
    with pytest.raises(ValueError):
        vie.problem_setup(op, torch.zeros(GRID, dtype=torch.float32), torch.zeros(GRID, dtype=torch.float64), e_inc,
                          298e6)
    with pytest.raises(ValueError):
        vie.field_gradient(op, e_inc, e_inc.to(torch.complex64), 298e6)
    x = torch.zeros((2, 3) + GRID, dtype=torch.complex128)
    assert "dtype" in _raises(vie.matvec_jm, op, op, x, _v(shape=GRID), _v(torch.complex64, GRID), 0.001, 298e6)
    assert "device tensor" in _raises(vie.matvec_jm, op, op, x, _v(shape=GRID), _v(shape=GRID), 0.001, 298e6)
    assert "dtype" in _raises(vie.solve_jm, op, op, x, _v(torch.complex64, GRID), _v(shape=GRID), 0.001, 298e6)


def test_numpy_inputs_are_refused():
    op = _FakeOp(N)
    x = _v()
    with pytest.raises(ValueError):
        vie.matvec(op, x, np.zeros(GRID, complex))


def test_piecewise_linear_calls_reject_mismatches():
    op = _FakeOp(N)
    x = _v(shape=(12,) + GRID)
    # the product checks the vectors' shape, then their device, then eps_c
    assert "contiguous" in _raises(vie.matvec_pwl, op, _v(shape=(11,) + GRID))
    assert "device tensor" in _raises(vie.matvec_pwl, op, x, _v(torch.complex64, GRID))
    assert "device tensor" in _raises(vie.matvec_pwl, op, x, kind="N")
    # several vectors: (nrhs, 12, n3, n2, n1)
    assert "device tensor" in _raises(vie.matvec_pwl, op, _v(shape=(2, 12) + GRID), kind="N")
    assert "b must be" in _raises(vie.solve_pwl, op, _v(shape=(3,) + GRID), _v(shape=GRID))
    assert "dtype" in _raises(vie.solve_pwl, op, x, _v(torch.complex64, GRID))
    xj = _v(shape=(2, 12) + GRID)
    assert "x must be" in _raises(vie.matvec_jm_pwl, op, op, _v(shape=(2, 3) + GRID), _v(shape=GRID),
                                  _v(shape=GRID), 0.001, 298e6)
    assert "dtype" in _raises(vie.matvec_jm_pwl, op, op, xj, _v(shape=GRID), _v(torch.complex64, GRID), 0.001, 298e6)
    assert "device tensor" in _raises(vie.matvec_jm_pwl, op, op, xj, _v(shape=GRID), _v(shape=GRID), 0.001, 298e6)
    assert "dtype" in _raises(vie.solve_jm_pwl, op, op, xj, _v(torch.complex64, GRID), _v(shape=GRID), 0.001, 298e6)
    assert "(10, 3" in _raises(vie.compress_pwl_k, np.zeros((10, 6) + GRID, complex))
