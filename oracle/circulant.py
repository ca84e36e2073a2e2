"""Circulant embedding and Fourier-domain Tucker factors (FP64).
Test infrastructure only.

The Toeplitz defining tensor of a Green's component covers offsets
D in [0, n1) x [0, n2) x [0, n3); offsets with negative entries follow from
the parity of the component: the xy, xz, yz components are odd along each of
their two axes, everything else is even.  The circulant embedding of length
L_i = 2 n_i per axis places offset -m at index L_i - m and leaves index n_i at
zero.  Because the embedding acts axis by axis it commutes with the Tucker
form: embedding the tensor equals embedding each factor column, and the same
holds for the FFT, so the Fourier-domain tensor is
G x1 F(E U1) x2 F(E U2) x3 F(E U3) (Sec. V-A).

FFT convention: forward unnormalised (exp(-2 pi i m k / L)), inverse scaled
by 1/L per axis.
"""
import numpy as np

from .tucker import tucker_reconstruct

# components xx, yy, zz, xy, xz, yz as (p, q)
COMPONENTS = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def component_index(p, q):
    p, q = min(p, q), max(p, q)
    return COMPONENTS.index((p, q))


def axis_signs(c):
    """Parity (+1 even, -1 odd) of component c along x, y, z."""
    p, q = COMPONENTS[c]
    return tuple(-1 if (p != q and a in (p, q)) else 1 for a in range(3))


def embed_columns(U, s):
    """Embed each column of U (n x r) to length 2n with parity s:
    e[m] = U[m] (m < n), e[n] = 0, e[2n - m] = s U[m] (1 <= m < n)."""
    U = np.asarray(U)
    n = U.shape[0]
    E = np.zeros((2 * n,) + U.shape[1:], dtype=np.complex128)
    E[:n] = U
    if n > 1:
        E[n + 1:] = s * U[1:][::-1]
    return E


def embed_tensor(A, signs):
    """Circulant embedding of a defining tensor A[i, j, k] to
    (2n1, 2n2, 2n3), axis by axis with the given parities."""
    E = np.asarray(A, dtype=np.complex128)
    for ax in range(3):
        E = np.moveaxis(embed_columns(np.moveaxis(E, ax, 0), signs[ax]), 0, ax)
    return E


def fourier_factor(U, s):
    """F(E U): DFT of the embedded factor columns (Sec. V-A)."""
    return np.fft.fft(embed_columns(U, s), axis=0)


def fourier_tensor_dense(A, signs):
    """3-D FFT of the circulant embedding of a dense defining tensor."""
    return np.fft.fftn(embed_tensor(A, signs))


def fourier_tensor_tucker(G, Us, signs):
    """Fourier-domain tensor from a Tucker form, reconstructed densely:
    G x1 F(E U1) x2 F(E U2) x3 F(E U3)."""
    Uh = [fourier_factor(U, s) for U, s in zip(Us, signs)]
    return tucker_reconstruct(G, Uh[0], Uh[1], Uh[2])
