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
