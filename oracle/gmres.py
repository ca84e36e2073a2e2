"""Restarted GMRES (FP64).  Test infrastructure only.

The paper solves the VIE system with GMRES at a relative tolerance, 50 inner
and 200 outer iterations (Sec. VI-C).  This is textbook GMRES(m): Arnoldi
with modified Gram-Schmidt plus one re-orthogonalisation pass, complex Givens
rotations for the least-squares problem, no preconditioner.  An Arnoldi
residual estimate at or below ``tol`` ends an inner cycle; the solve stops
only when the true residual ||b - A x|| / ||b||, recomputed at every restart,
is at or below ``tol``.
"""
import numpy as np


class GmresInfo:
    def __init__(self):
        self.matvecs = 0
        self.restarts = 0
        self.converged = False
        self.rel_residual = np.inf
        self.history = []          # true relative residual at each restart


def _givens(a, b):
    """Complex rotation (c real, s complex) with [c s; -conj(s) c][a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0
    if a == 0:
        return 0.0, 1.0
    t = np.hypot(abs(a), abs(b))
    c = abs(a) / t
    s = (a / abs(a)) * np.conj(b) / t
    return c, s


def gmres(apply_A, b, x0=None, tol=1e-6, restart=50, max_outer=200):
    """Solve A x = b; ``apply_A`` maps a flat complex128 vector to A x."""
    b = np.asarray(b, dtype=np.complex128).ravel()
    n = b.size
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128).ravel()
    info = GmresInfo()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        info.converged = True
        info.rel_residual = 0.0
        return np.zeros_like(b), info
    m = int(restart)
    for outer in range(max_outer + 1):
        r = b - apply_A(x)
        info.matvecs += 1
        beta = np.linalg.norm(r)
        rel = beta / bnorm
        info.history.append(rel)
        info.rel_residual = rel
        if rel <= tol:
            info.converged = True
            return x, info
        if outer == max_outer:
            break
        info.restarts = outer
        V = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            w = apply_A(V[j])
            info.matvecs += 1
            for _ in range(2):                  # MGS, then one re-orthogonalisation
                for i in range(j + 1):
                    h = np.vdot(V[i], w)
                    H[i, j] += h
                    w = w - h * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):                  # previous rotations on column j
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            a, bb = H[j, j], H[j + 1, j]
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            breakdown = abs(H[j, j]) == 0.0 or np.linalg.norm(w) == 0.0
            if abs(g[j + 1]) / bnorm <= tol or breakdown:
                break
            V[j + 1] = w / np.linalg.norm(w)
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):          # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + V[:k].T @ y
    return x, info
