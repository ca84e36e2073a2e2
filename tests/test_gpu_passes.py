"""Single passes of the device matvec against the oracle's five-pass split
(Sec. V-A), through the debug entry points of the C ABI.

* vie_debug_pad / vie_debug_crop (the X+ and X- kernels with the identity in
  place of the FFT): the zero padding and transposes are bit-exact against
  the index maps, and crop(pad(x)) = x bitwise, at register-FFT lengths
  L1 = 128, 192, 224, 256, 512 and mixed-radix lengths;
* every pass on integer data with n_i in {1, 2} (FFT lengths 2 and 4: twiddles
  +-1, +-i, all arithmetic exact) equals the oracle's pass bit for bit, the
  z pass with an integer Tucker form, in all four modes;
* every pass at register-FFT lengths against the oracle's pass on the same
  (the oracle's) Tucker form (relative 1e-6 complex64, 1e-13 complex128);
* the five debug passes in sequence equal vie_matvec bitwise."""
import itertools

import numpy as np
import pytest
import torch

import vie_inputs as vi
from gpu_common import K0, say, to_dev
from oracle import circulant, operator as opm, passes
from paper_1811_00484_amd import vie

pytestmark = pytest.mark.gpu

DTYPES = [torch.complex64, torch.complex128]


def _icx(rng, shape):
    return rng.integers(-3, 4, shape) + 1j * rng.integers(-3, 4, shape)


def _np(t):
    return t.cpu().numpy().astype(np.complex128)


def _small_operator(n, tol=1e-6, h=0.005):
    return vie.compress(vi.green_tensor(n, h, K0), tol=tol)


PAD_GRIDS = [(64, 5, 3), (96, 7, 2), (112, 3, 4), (128, 9, 2), (256, 2, 3), (5, 7, 3), (48, 4, 2), (1, 3, 2)]


@pytest.mark.parametrize("n", PAD_GRIDS)
@pytest.mark.parametrize("dt", DTYPES)
def test_pad_and_crop_are_bit_exact(n, dt):
    say("   pad/crop", n, dt)
    op = _small_operator(n)
    n1, n2, n3 = n
    rng = np.random.default_rng(sum(n))
    x = rng.standard_normal((2, 3, n3, n2, n1)) + 1j * rng.standard_normal((2, 3, n3, n2, n1))
    xd = to_dev(x, dt)
    s1 = vie.debug_pad(op, xd)
    expect = np.zeros((2, 3, n3, 2 * n1, n2), complex)
    expect[:, :, :, :n1, :] = np.swapaxes(_np(xd), 3, 4)
    assert np.array_equal(_np(s1), expect)
    y = vie.debug_crop(op, s1)
    assert torch.equal(y, xd)
    s3 = rng.standard_normal(expect.shape) + 1j * rng.standard_normal(expect.shape)
    s3d = to_dev(s3, dt)
    yc = vie.debug_crop(op, s3d)
    assert np.array_equal(_np(yc), np.swapaxes(_np(s3d)[:, :, :, :n1, :], 3, 4))


def _integer_op(n, seed):
    rng = np.random.default_rng(seed)
    cores, factors = [], []
    for c in range(6):
        signs = circulant.axis_signs(c)
        r = [int(rng.integers(1, min(n[a], 2) + 1)) for a in range(3)]
        G = rng.integers(-1, 2, r) + 1j * rng.integers(-1, 2, r)
        Us = []
        for a in range(3):
            U = rng.integers(-1, 2, (n[a], r[a])) + 1j * rng.integers(-1, 2, (n[a], r[a]))
            if signs[a] < 0:
                U[0, :] = 0
            Us.append(U)
        cores.append(G)
        factors.append(Us)
    nhat = [circulant.fourier_tensor_tucker(cores[c], factors[c], circulant.axis_signs(c)) for c in range(6)]
    return vie.from_tucker(n, cores, factors), opm.FourierOperator(n, nhat)


def _oracle_form_on_device(ref):
    """The oracle's own HOSVD Tucker form uploaded with vie_op_from_tucker,
    so that both sides apply the same operator (two HOSVD implementations
    at tol 1e-6 give forms that differ far above the complex128 rounding);
    the factor rows at offset 0 of odd axes, zero up to rounding, are set to
    exact zeros as the upload requires."""
    factors = []
    for c in range(6):
        signs = circulant.axis_signs(c)
        Us = [U.copy() for U in ref.factors[c]]
        for a in range(3):
            if signs[a] < 0:
                Us[a][0, :] = 0
        factors.append(Us)
    return vie.from_tucker(ref.n, ref.cores, factors)


@pytest.mark.parametrize("n", list(itertools.product((1, 2), repeat=3)))
@pytest.mark.parametrize("dt", DTYPES)
def test_each_pass_is_bit_exact_on_integer_data(n, dt):
    op, ref = _integer_op(n, 40 + sum(n))
    n1, n2, n3 = n
    rng = np.random.default_rng(9)
    x = _icx(rng, (1, 3, n3, n2, n1))
    eps = rng.integers(1, 4, (n3, n2, n1)) - 1j * rng.integers(0, 3, (n3, n2, n1))
    xd, ed = to_dev(x, dt), to_dev(eps, dt)
    for mode in ("A", "AH", "N", "NH"):
        kind, adj = ("N" if mode[0] == "N" else "A"), mode.endswith("H")
        s1 = passes.pass_x_forward(x, eps, mode)
        s1d = vie.debug_pass(op, 0, x=xd, eps_c=ed, kind=kind, adjoint=adj)
        assert np.array_equal(_np(s1d), s1), (n, mode, 0)
        s2 = passes.pass_y_forward(s1)
        s2d = vie.debug_pass(op, 1, inp=to_dev(s1, dt), kind=kind, adjoint=adj)
        assert np.array_equal(_np(s2d), s2), (n, mode, 1)
        s2z = passes.pass_z(s2, ref.nhat, conj=adj)
        s2zd = vie.debug_pass(op, 2, inp=to_dev(s2, dt), kind=kind, adjoint=adj)
        assert np.array_equal(_np(s2zd), s2z), (n, mode, 2)
        s3 = passes.pass_y_inverse(s2z, n2)
        s3d = vie.debug_pass(op, 3, inp=to_dev(s2z, dt), kind=kind, adjoint=adj)
        assert np.array_equal(_np(s3d), s3), (n, mode, 3)
        y = passes.pass_x_inverse(s3, n1, x, eps, mode)
        yd = vie.debug_pass(op, 4, inp=to_dev(s3, dt), x=xd, eps_c=ed, kind=kind, adjoint=adj)
        assert np.array_equal(_np(yd), y), (n, mode, 4)


REG_GRIDS = [(64, 64, 64), (96, 112, 20), (112, 8, 128), (256, 6, 5), (12, 256, 9), (10, 9, 256)]


@pytest.mark.parametrize("n", REG_GRIDS)
@pytest.mark.parametrize("dt", DTYPES)
def test_each_pass_matches_the_oracle_at_register_fft_lengths(n, dt):
    say("   passes", n, dt)
    G = vi.green_tensor(n, 0.004, K0)
    ref = opm.tucker_operator(G, 1e-6)
    op = _oracle_form_on_device(ref)
    n1, n2, n3 = n
    rng = np.random.default_rng(sum(n) + 1)
    x = rng.standard_normal((1, 3, n3, n2, n1)) + 1j * rng.standard_normal((1, 3, n3, n2, n1))
    eps = 1 + rng.uniform(0, 50, (n3, n2, n1)) - 1j * rng.uniform(0, 30, (n3, n2, n1))
    tol = 1e-6 if dt == torch.complex64 else 1e-13
    xd, ed = to_dev(x, dt), to_dev(eps, dt)

    def close(a, b, what):
        err = float(np.linalg.norm(a - b) / np.linalg.norm(b))
        say("     ", what, "%.2e" % err)
        assert err <= tol, what

    for mode in ("A", "AH"):
        adj = mode == "AH"
        s1 = passes.pass_x_forward(x, eps, mode)
        close(_np(vie.debug_pass(op, 0, x=xd, eps_c=ed, adjoint=adj)), s1, "X+ " + mode)
        s2 = passes.pass_y_forward(s1)
        close(_np(vie.debug_pass(op, 1, inp=to_dev(s1, dt))), s2, "Y+")
        s2z = passes.pass_z(s2, ref.nhat, conj=adj)
        close(_np(vie.debug_pass(op, 2, inp=to_dev(s2, dt), adjoint=adj)), s2z, "Z " + mode)
        s3 = passes.pass_y_inverse(s2z, n2)
        close(_np(vie.debug_pass(op, 3, inp=to_dev(s2z, dt))), s3, "Y-")
        y = passes.pass_x_inverse(s3, n1, x, eps, mode)
        close(_np(vie.debug_pass(op, 4, inp=to_dev(s3, dt), x=xd, eps_c=ed, adjoint=adj)), y, "X- " + mode)


@pytest.mark.parametrize("n", [(64, 64, 64), (20, 15, 18)])
@pytest.mark.parametrize("dt", DTYPES)
def test_debug_passes_in_sequence_equal_the_matvec_bitwise(n, dt):
    op = _small_operator(n)
    n1, n2, n3 = n
    rng = np.random.default_rng(3)
    x = to_dev(rng.standard_normal((2, 3, n3, n2, n1)) + 1j * rng.standard_normal((2, 3, n3, n2, n1)), dt)
    e = to_dev(1 + rng.uniform(0, 50, (n3, n2, n1)) - 1j * rng.uniform(0, 30, (n3, n2, n1)), dt)
    for adj in (False, True):
        s = vie.debug_pass(op, 0, x=x, eps_c=e, adjoint=adj)
        s = vie.debug_pass(op, 1, inp=s)
        s = vie.debug_pass(op, 2, inp=s, out=s, adjoint=adj)
        s = vie.debug_pass(op, 3, inp=s)
        y = vie.debug_pass(op, 4, inp=s, x=x, eps_c=e, adjoint=adj)
        assert torch.equal(y, vie.matvec(op, x, e, adjoint=adj))


def test_debug_pass_argument_errors():
    op = _small_operator((6, 5, 4))
    x = to_dev(np.zeros((1, 3, 4, 5, 6), complex), torch.complex64)
    lib = vie.load()
    s = vie._stream()
    # x required by pass 0; in required by pass 1; bad pass number; bad kind
    assert lib.vie_debug_pass(op.handle, 0, 0, 0, 0, 0, None, None, None, x.data_ptr(), 1, s) == vie.VIE_E_ARG
    assert lib.vie_debug_pass(op.handle, 1, 0, 0, 0, 0, None, None, None, x.data_ptr(), 1, s) == vie.VIE_E_ARG
    assert lib.vie_debug_pass(op.handle, 5, 0, 0, 0, 0, None, x.data_ptr(), None, x.data_ptr(), 1, s) == vie.VIE_E_ARG
    assert lib.vie_debug_pass(op.handle, 0, 7, 0, 0, 0, None, x.data_ptr(), None, x.data_ptr(), 1, s) == vie.VIE_E_ARG
    # output overlapping the input
    assert lib.vie_debug_pad(op.handle, 0, x.data_ptr(), x.data_ptr(), 1, s) == vie.VIE_E_ARG
