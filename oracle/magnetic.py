"""The magnetic operator K of eq. 5 and the b1+ observable of eq. 18 (FP64).
Test infrastructure only.

K is the curl of the single-layer potential.  With piecewise-constant
current coefficients and Galerkin rows divided by the voxel volume its
defining tensor is antisymmetric in the component pair (Kt_qp = -Kt_pq, zero
diagonal): three unique components xy, xz, yz, stored like the N tensor for
offsets D in [0, n1) x [0, n2) x [0, n3) with the observation voxel at D and
the source voxel at 0, so that

    (K u)_p(m) = h sum_q sum_m' Kt_pq(m - m') u_q(m')

is a 3-level Toeplitz convolution (Sec. II-B).  Each component is the
derivative of an even function along one axis: Kt_xy is odd along z, Kt_xz
along y, Kt_yz along x, and even along the other two.  The FFT evaluation
embeds each component with these parities (Sec. V-A), and the 3x3 product in
the Fourier domain uses the antisymmetric pattern.

The full JMVIE operator of eq. 4 (``jm_matvec``) couples the electric and
magnetic polarisation currents J and M through K, with a magnetic contrast
chi_h = mu_c - 1 beside the electric one.

Observables: H = H_inc + K J for the polarisation current J of the electric
equation (u = J, eq. 3; the tissue is non-magnetic, so M = 0 in eq. 1 and
the second block row only produces the field), and |b1+| = mu0 |H_x + i H_y|
(eq. 18).
"""
import numpy as np
import scipy.fft as sfft

from vie_inputs.constants import MU0

from .circulant import fourier_tensor_dense, fourier_tensor_tucker
from .operator import FourierOperator, _workers
from .tucker import from_storage, hosvd, to_storage

# stored components as (p, q) with p < q
K_COMPONENTS = ((0, 1), (0, 2), (1, 2))
# the axis each component is odd along: d/dz for xy, d/dy for xz, d/dx for yz
K_ODD_AXIS = (2, 1, 0)


def k_axis_signs(c):
    """Parity (+1 even, -1 odd) of K component c (xy, xz, yz) along x, y, z."""
    return tuple(-1 if a == K_ODD_AXIS[c] else 1 for a in range(3))


def k_entry(kt, p, q, D):
    """Kt_pq at a signed offset D = (dx, dy, dz): zero on the diagonal,
    antisymmetric in (p, q), odd along the component's derivative axis."""
    if p == q:
        return 0j
    sign = 1
    if p > q:
        p, q = q, p
        sign = -1
    c = K_COMPONENTS.index((p, q))
    s = k_axis_signs(c)
    for a in range(3):
        if D[a] < 0:
            sign *= s[a]
    return sign * kt[c, abs(D[2]), abs(D[1]), abs(D[0])]


def brute_force_K(kt, u):
    """sum_q sum_m' Kt_pq(m - m') u_q(m') written out (tiny grids); no h."""
    n3, n2, n1 = u.shape[1:]
    out = np.zeros_like(u, dtype=np.complex128)
    idx = [(i, j, k) for k in range(n3) for j in range(n2) for i in range(n1)]
    for p in range(3):
        for (i, j, k) in idx:
            acc = 0j
            for q in range(3):
                for (i2, j2, k2) in idx:
                    acc += k_entry(kt, p, q, (i - i2, j - j2, k - k2)) * u[q, k2, j2, i2]
            out[p, k, j, i] = acc
    return out


def dense_matrix_K(kt):
    """Explicit 3V x 3V matrix of sum_q Kt_pq(m - m') (tiny grids), unknown
    ordering (q, k, j, i) as in the storage layout."""
    n3, n2, n1 = kt.shape[1:]
    V = n1 * n2 * n3
    idx = [(i, j, k) for k in range(n3) for j in range(n2) for i in range(n1)]
    M = np.zeros((3 * V, 3 * V), dtype=np.complex128)
    for p in range(3):
        for q in range(3):
            for a, (i, j, k) in enumerate(idx):
                for b, (i2, j2, k2) in enumerate(idx):
                    M[p * V + a, q * V + b] = k_entry(kt, p, q, (i - i2, j - j2, k - k2))
    return M


def dense_k_operator(kt):
    """Fourier-domain tensors of the three dense K components."""
    n = (kt.shape[3], kt.shape[2], kt.shape[1])
    nhat = [fourier_tensor_dense(from_storage(kt[c]), k_axis_signs(c)) for c in range(3)]
    return FourierOperator(n, nhat)


def tucker_k_operator(kt, tol, rule=0):
    """HOSVD of each K component (Alg. 1), Fourier-domain tensor from the
    Tucker form with the K parities (Sec. V-A)."""
    n = (kt.shape[3], kt.shape[2], kt.shape[1])
    nhat, ranks, factors, cores = [], [], [], []
    for c in range(3):
        G, Us, _ = hosvd(from_storage(kt[c]), tol, rule)
        nhat.append(fourier_tensor_tucker(G, Us, k_axis_signs(c)))
        ranks.append(tuple(U.shape[1] for U in Us))
        factors.append(Us)
        cores.append(G)
    return FourierOperator(n, nhat, ranks, factors, cores)


def apply_K(op, u):
    """sum_q Kt_pq * u_q (no h) by zero padding to (2n1, 2n2, 2n3), FFT, the
    antisymmetric 3x3 product in the Fourier domain, inverse FFT, crop."""
    n1, n2, n3 = op.n
    L = (2 * n1, 2 * n2, 2 * n3)
    w = _workers()
    Xh = []
    for q in range(3):
        pad = np.zeros(L, dtype=np.complex128)
        pad[:n1, :n2, :n3] = from_storage(u[q])
        Xh.append(sfft.fftn(pad, workers=w))
    Kxy, Kxz, Kyz = op.nhat
    Yh = (Kxy * Xh[1] + Kxz * Xh[2],
          -Kxy * Xh[0] + Kyz * Xh[2],
          -Kxz * Xh[0] - Kyz * Xh[1])
    out = np.empty((3, n3, n2, n1), dtype=np.complex128)
    for p in range(3):
        out[p] = to_storage(sfft.ifftn(Yh[p], workers=w)[:n1, :n2, :n3])
    return out


def magnetic_field(op, u, h_inc, h):
    """H = H_inc + K J with J = u (physical K = h Kt)."""
    return h_inc + h * apply_K(op, u)


def b1_plus(H):
    """|b1+| = mu0 |H_x + i H_y| (eq. 18)."""
    return MU0 * np.abs(H[0] + 1j * H[1])


def jm_matvec(op_n, op_k, eps_c, mu_c, x, h, freq_hz):
    """The full JMVIE operator of eq. 4 on x = [J; M] (shape (2, 3, n3, n2, n1)):

        y_J = eps_c J - chi_e N J + c_e chi_e K M
        y_M = mu_c M - chi_h N M - c_m chi_h K J

    with chi_e = eps_c - 1, chi_h = mu_c - 1, c_e = i omega eps0,
    c_m = i omega mu0 (eq. 2) and the physical K = h Kt."""
    from vie_inputs.constants import EPS0, omega

    from .operator import apply_N
    ce = 1j * omega(freq_hz) * EPS0
    cm = 1j * omega(freq_hz) * MU0
    chi_e = np.asarray(eps_c) - 1.0
    chi_h = np.asarray(mu_c) - 1.0
    J, M = x[0], x[1]
    yJ = eps_c[None] * J - chi_e[None] * apply_N(op_n, J) + ce * h * chi_e[None] * apply_K(op_k, M)
    yM = mu_c[None] * M - chi_h[None] * apply_N(op_n, M) - cm * h * chi_h[None] * apply_K(op_k, J)
    return np.stack([yJ, yM])


def jm_rhs(eps_c, mu_c, e_inc, h_inc, freq_hz):
    """Right-hand side of eq. 1: [c_e chi_e E_inc; c_m chi_h H_inc]."""
    from vie_inputs.constants import EPS0, omega
    ce = 1j * omega(freq_hz) * EPS0
    cm = 1j * omega(freq_hz) * MU0
    return np.stack([ce * (np.asarray(eps_c) - 1.0)[None] * e_inc, cm * (np.asarray(mu_c) - 1.0)[None] * h_inc])


def solve_jm(op_n, op_k, eps_c, mu_c, b, h, freq_hz, tol=1e-8, restart=50, max_outer=200):
    """GMRES on the full JMVIE system of eq. 4 (the oracle's GMRES)."""
    from .gmres import gmres
    shape = b.shape

    def A(v):
        return jm_matvec(op_n, op_k, eps_c, mu_c, v.reshape(shape), h, freq_hz).ravel()

    x, info = gmres(A, b, tol=tol, restart=restart, max_outer=max_outer)
    return x.reshape(shape), info
