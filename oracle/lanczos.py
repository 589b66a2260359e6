"""Plain Lanczos for the lowest eigenpair of a symmetric operator.

Full reorthogonalisation, no restarts; stops when the residual 2-norm of the
normalised Ritz vector falls below ``tol``.  The local problems of the
additive two-level method are solved with Lanczos in the paper's experiments
(Section 4); this is the textbook recurrence.
"""
from __future__ import annotations

import numpy as np


def lanczos_lowest(matvec, v0: np.ndarray, tol: float = 1e-10, maxiter: int = 500):
    n = v0.size
    q = v0 / np.linalg.norm(v0)
    Q = [q]
    alphas, betas = [], []
    theta, u = None, q
    for it in range(min(maxiter, n)):
        w = matvec(Q[-1])
        a = float(Q[-1] @ w)
        w = w - a * Q[-1] - (betas[-1] * Q[-2] if betas else 0.0)
        Qm = np.array(Q)
        w -= Qm.T @ (Qm @ w)
        w -= Qm.T @ (Qm @ w)
        alphas.append(a)
        T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
        ev, evec = np.linalg.eigh(T)
        theta = ev[0]
        u = Qm.T @ evec[:, 0]
        b = float(np.linalg.norm(w))
        res = abs(b * evec[-1, 0])
        if res <= tol or b < 1e-14:
            break
        betas.append(b)
        Q.append(w / b)
    u = u / np.linalg.norm(u)
    return theta, u
