"""Pin of the oracle's adjoint gradient: central finite differences of the
objective through tightly converged FP64 solves."""
import numpy as np

import vie_inputs as vi
from oracle import gradient, operator as opm, physics

F = 298e6
K0 = vi.wavenumber(F)


def test_adjoint_gradient_matches_central_differences():
    n = (6, 5, 7)
    h = 0.004
    er, sg, label = vi.head_phantom(n, h * 4.0, seed=3)   # head scaled into a small box
    epsc = vi.complex_permittivity(er, sg, F)
    e = vi.dipole_field(n, h, F, (0.03, 0.0, 0.0), np.ones(er.shape, bool))
    op = opm.dense_operator(vi.green_tensor(n, h, K0))
    rng = np.random.default_rng(50)
    tissue = np.nonzero(label.ravel() >= 0)[0]
    targets = rng.choice(tissue, 10, replace=False)
    u, _ = physics.solve_currents(op, epsc, e, F, tol=1e-13)
    E0 = physics.total_field(op, u, e, F)
    E_target = E0[0].ravel()[targets] * (1.0 + 0.1 * rng.standard_normal(10))
    L, g_eps, g_sig, _ = gradient.adjoint_gradient(op, epsc, e, F, targets, E_target, tol=1e-13)

    def objective(er_, sg_):
        ec = vi.complex_permittivity(er_, sg_, F)
        uu, _ = physics.solve_currents(op, ec, e, F, tol=1e-13)
        return gradient.objective(physics.total_field(op, uu, e, F), targets, E_target)

    picks = rng.choice(tissue, 6, replace=False)
    fd_e, fd_s, ad_e, ad_s = [], [], [], []
    for v in picks:
        idx = np.unravel_index(v, er.shape)
        for which in ("eps", "sig"):
            base = er if which == "eps" else sg
            step = 1e-4 * base[idx]
            p = base.copy(); p[idx] += step
            m = base.copy(); m[idx] -= step
            if which == "eps":
                d = (objective(p, sg) - objective(m, sg)) / (2 * step)
                fd_e.append(d); ad_e.append(g_eps[idx])
            else:
                d = (objective(er, p) - objective(er, m)) / (2 * step)
                fd_s.append(d); ad_s.append(g_sig[idx])
    fd = np.array(fd_e + fd_s)
    ad = np.array(ad_e + ad_s)
    assert np.linalg.norm(ad - fd) <= 1e-5 * np.linalg.norm(fd)
