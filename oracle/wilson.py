"""Wilson-Dirac matrix A = I - kappa D (the complex non-Hermitian operator of
Example 7; the paper names it but does not write it out, so the textbook
definition is used).

  (D psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu)
                      + (1 + gamma_mu) U_mu(x - mu)^H psi(x - mu) ]

with psi picking up the factor bc[mu] (= -1 for antiperiodic time) when a hop
wraps around the lattice in direction mu. The shifted systems of eq. (1.1)
use (A - sigma I) psi = (1 - sigma) psi - kappa D psi.

Gamma matrices: a chiral basis (Hermitian, {g_mu, g_nu} = 2 delta_{mu nu},
gamma5 = g1 g2 g3 g4 = diag(1, 1, -1, -1)). The paper does not fix a basis;
this one is a reading, and every result below (spectrum, gamma5-hermiticity,
gauge covariance) is basis independent.

Layouts are the canonical ones of ``synth``: psi [..., t, z, y, x, spin, colour]
(a leading batch axis is allowed) and links [mu, t, z, y, x, a, b].
"""
import numpy as np

I4 = np.eye(4, dtype=np.complex128)
GAMMA = np.array([
    [[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]

# psi axes counted from the end: x=-3, y=-4, z=-5, t=-6; links mu axes 0..3
# are [t, z, y, x] so direction mu lives on link axis 3 - mu.
_PSI_AXIS = (-3, -4, -5, -6)


def _shift(a, mu, step, bc, axis):
    """a(x + step*mu) with the boundary factor on the wrapped slice."""
    out = np.roll(a, -step, axis=axis)
    if bc[mu] != 1:
        n = a.shape[axis]
        idx = [slice(None)] * a.ndim
        idx[axis] = n - 1 if step > 0 else 0
        out[tuple(idx)] *= bc[mu]
    return out


def hop(links, psi, bc=(1, 1, 1, -1)):
    """D psi (the hopping term), for psi of shape [..., t, z, y, x, 4, 3].

    Colour: (U psi)_sa = sum_b U_ab psi_sb, written psi @ U^T; the backward
    term U^H psi is psi @ conj(U). Spin: (1 -/+ gamma_mu) @ psi."""
    out = np.zeros_like(psi)
    for mu in range(4):
        ax = _PSI_AXIS[mu]
        u = links[mu]
        fwd = _shift(psi, mu, +1, bc, ax)
        upsi = np.matmul(fwd, np.swapaxes(u, -1, -2))
        out += np.matmul(I4 - GAMMA[mu], upsi)
        ub = np.roll(u, 1, axis=3 - mu)          # U_mu(x - mu)
        bwd = _shift(psi, mu, -1, bc, ax)
        udpsi = np.matmul(bwd, ub.conj())
        out += np.matmul(I4 + GAMMA[mu], udpsi)
    return out


def apply_A(links, kappa, psi, sigma=0.0, bc=(1, 1, 1, -1)):
    """(A - sigma I) psi = (1 - sigma) psi - kappa D psi."""
    return (1.0 - sigma) * psi - kappa * hop(links, psi, bc)


class WilsonOperator:
    """Flat-vector view of A for the Krylov routines (n = 12 V unknowns)."""

    def __init__(self, links, kappa, bc=(1, 1, 1, -1)):
        self.links = links
        self.kappa = kappa
        self.bc = tuple(bc)
        lt, lz, ly, lx = links.shape[1:5]
        self.dims = (lx, ly, lz, lt)
        self.shape = (lt, lz, ly, lx, 4, 3)
        self.n = 12 * lx * ly * lz * lt
        self.count = 0

    def __call__(self, v):
        """A v for a flat vector (or a batch [nb, n])."""
        self.count += 1 if v.ndim == 1 else v.shape[0]
        psi = v.reshape(v.shape[:-1] + self.shape)
        return apply_A(self.links, self.kappa, psi, 0.0, self.bc).reshape(v.shape)

    def shifted(self, v, sigma):
        return self(v) - sigma * v

    def hop_flat(self, v):
        psi = v.reshape(v.shape[:-1] + self.shape)
        return hop(self.links, psi, self.bc).reshape(v.shape)


def dense_hop(links, bc=(1, 1, 1, -1), chunk=512):
    """D as a dense matrix, assembled column by column from ``hop``."""
    lt, lz, ly, lx = links.shape[1:5]
    n = 12 * lx * ly * lz * lt
    shape = (lt, lz, ly, lx, 4, 3)
    mat = np.zeros((n, n), dtype=np.complex128)
    for s in range(0, n, chunk):
        e = np.zeros((min(chunk, n - s), n), dtype=np.complex128)
        e[np.arange(e.shape[0]), s + np.arange(e.shape[0])] = 1
        mat[:, s:s + e.shape[0]] = hop(links, e.reshape((-1,) + shape), bc).reshape(e.shape[0], n).T
    return mat


def dense_hop_from_definition(links, bc=(1, 1, 1, -1)):
    """D assembled directly from its definition with explicit site loops and
    Kronecker blocks (1 -/+ gamma_mu) (x) U; used to pin ``hop``."""
    lt, lz, ly, lx = links.shape[1:5]
    ext = (lx, ly, lz, lt)
    vol = lx * ly * lz * lt
    mat = np.zeros((12 * vol, 12 * vol), dtype=np.complex128)

    def lex(c):
        return c[0] + lx * (c[1] + ly * (c[2] + lz * c[3]))

    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    here = (x, y, z, t)
                    i = lex(here)
                    for mu in range(4):
                        up = list(here)
                        up[mu] += 1
                        fsign = 1.0
                        if up[mu] == ext[mu]:
                            up[mu] = 0
                            fsign = bc[mu]
                        dn = list(here)
                        dn[mu] -= 1
                        bsign = 1.0
                        if dn[mu] < 0:
                            dn[mu] = ext[mu] - 1
                            bsign = bc[mu]
                        u_here = links[mu, t, z, y, x]
                        u_dn = links[mu, dn[3], dn[2], dn[1], dn[0]]
                        j = lex(up)
                        mat[12 * i:12 * i + 12, 12 * j:12 * j + 12] += \
                            fsign * np.kron(I4 - GAMMA[mu], u_here)
                        j = lex(dn)
                        mat[12 * i:12 * i + 12, 12 * j:12 * j + 12] += \
                            bsign * np.kron(I4 + GAMMA[mu], u_dn.conj().T)
    return mat


def free_field_eigenvalues(dims, bc=(1, 1, 1, -1)):
    """Closed-form spectrum of D with unit links: for each lattice momentum p
    (p_mu = 2 pi n / L, or pi (2n+1) / L for an antiperiodic direction) the
    eigenvalues are 2 sum cos p_mu +/- 2i sqrt(sum sin^2 p_mu), each 6 times
    (2 spin x 3 colour)."""
    grids = []
    for mu, L in enumerate(dims):
        nn = np.arange(L)
        grids.append(2 * np.pi * nn / L if bc[mu] == 1 else np.pi * (2 * nn + 1) / L)
    p = np.meshgrid(*grids, indexing="ij")
    re = 2 * sum(np.cos(q) for q in p).ravel()
    im = 2 * np.sqrt(sum(np.sin(q) ** 2 for q in p)).ravel()
    ev = np.concatenate([re + 1j * im, re - 1j * im])
    return np.repeat(ev, 6)


def gamma5_flat(v, shape):
    """gamma5 applied on the spin index of a flat vector."""
    psi = v.reshape(shape)
    return np.einsum("st,...tc->...sc", GAMMA5, psi).reshape(v.shape)
