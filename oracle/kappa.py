"""The critical hopping parameter of the synthetic operator family.

Example 7 runs at kappa approximately kappa_critical. Here kappa_c is read as
the largest kappa > 0 for which every eigenvalue of I - kappa D has positive
real part; since Re(1 - kappa lambda) = 1 - kappa Re(lambda), that is
kappa_c = 1 / lambda_R with lambda_R = max Re lambda(D).

lambda_R is taken from a dense eigensolve for small n and from ARPACK
(which='LR') otherwise; ``bisect_kappa_c`` re-derives kappa_c from the same
eigenvalues by bisection on the positivity predicate, as a cross-check.
"""
import numpy as np
import scipy.sparse.linalg as sla

from . import wilson


def rightmost_dense(links, bc=(1, 1, 1, -1)):
    ev = np.linalg.eigvals(wilson.dense_hop(links, bc))
    return ev


def rightmost_arpack(links, bc=(1, 1, 1, -1), nev=6, ncv=64, tol=1e-8, seed=7, maxiter=None):
    lt, lz, ly, lx = links.shape[1:5]
    n = 12 * lx * ly * lz * lt
    shape = (lt, lz, ly, lx, 4, 3)

    def mv(v):
        v = np.asarray(v, dtype=np.complex128).ravel()
        return wilson.hop(links, v.reshape(shape), bc).ravel()

    op = sla.LinearOperator((n, n), matvec=mv, dtype=np.complex128)
    v0 = np.random.default_rng(seed).standard_normal(n) + 0j
    ev = sla.eigs(op, k=nev, which="LR", ncv=ncv, tol=tol, v0=v0, maxiter=maxiter,
                  return_eigenvectors=False)
    return ev


def rightmost_restarted_arnoldi(links, bc=(1, 1, 1, -1), m=60, restarts=6, seed=7):
    """Rightmost eigenvalue of D by explicitly restarted Arnoldi: m Arnoldi
    steps (CGS2), take the Ritz pair of largest real part, restart from its
    Ritz vector. Returns (Ritz values of the last cycle, Ritz residual norm
    ||D y - theta y|| of the kept pair with ||y|| = 1)."""
    lt, lz, ly, lx = links.shape[1:5]
    n = 12 * lx * ly * lz * lt
    shape = (lt, lz, ly, lx, 4, 3)

    def mv(v):
        return wilson.hop(links, v.reshape(shape), bc).ravel()

    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    theta = None
    res = None
    for _ in range(restarts):
        V[:] = 0
        H[:] = 0
        V[:, 0] = v
        for j in range(m):
            w = mv(V[:, j])
            for _ in range(2):
                h = V[:, :j + 1].conj().T @ w
                w = w - V[:, :j + 1] @ h
                H[:j + 1, j] += h
            H[j + 1, j] = np.linalg.norm(w)
            V[:, j + 1] = w / H[j + 1, j]
        theta, g = np.linalg.eig(H[:m, :m])
        i = int(np.argmax(theta.real))
        y = V[:, :m] @ g[:, i]
        y /= np.linalg.norm(y)
        res = np.linalg.norm(mv(y) - theta[i] * y)
        v = y
    return theta, res


def kappa_c_from_eigs(ev):
    return 1.0 / np.max(ev.real)


def bisect_kappa_c(ev, rel=1e-12):
    """sup{kappa > 0 : min Re(1 - kappa lambda) > 0} by bisection."""
    def ok(kap):
        return np.min(1.0 - kap * ev.real) > 0

    lo, hi = 0.0, 1.0
    while ok(hi):
        hi *= 2
    while hi - lo > rel * hi:
        mid = 0.5 * (lo + hi)
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo
