"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the solver. It only draws the data the
problem (A - sigma_i I) x_i^j = b^j is posed on (Sec. 1, eq. (1.1)):

* gauge links U_mu(x) = exp(i * eps * H_mu(x)) with H a traceless Hermitian
  Gaussian matrix (the paper's QCD configuration of Example 7 is not
  available; these synthetic fields stand in for it),
* right-hand sides: complex Gaussian or Z4 noise vectors (Example 7 notes
  that in QCD the right-hand sides are noise vectors),
* the table of workloads (lattice sizes, shifts, restart parameters),
* the hopping parameter kappa of each workload, read from ``manifest.json``.
  That file is written by ``oracle/make_manifest.py`` (the oracle bisects
  kappa_c); nothing here computes it.

Canonical layouts (complex128, C order):
  links  [mu=x,y,z,t][t][z][y][x][a][b],  U_mu(x) multiplies psi(x + mu)
  vector [t][z][y][x][spin 4][colour 3]
"""
import json
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
MANIFEST = os.path.join(_HERE, "manifest.json")


def _gell_mann():
    """The eight Gell-Mann matrices (standard normalisation tr(l_a l_b) = 2 delta)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


GELL_MANN = _gell_mann()


def gauge_links(dims, eps, seed, chunk=1 << 18):
    """Random SU(3) links U = exp(i eps H), H = sum_a w_a lambda_a / 2, w ~ N(0,1).

    dims = (Lx, Ly, Lz, Lt). The Gaussian draws are taken in one call,
    ``default_rng(seed).standard_normal((4, Lt, Lz, Ly, Lx, 8))``, so the field
    is a fixed function of (dims, eps, seed). The exponential is taken through
    the eigendecomposition of the Hermitian H, in chunks to bound memory.
    """
    lx, ly, lz, lt = dims
    w = np.random.default_rng(seed).standard_normal((4, lt, lz, ly, lx, 8))
    w = w.reshape(-1, 8)
    out = np.empty((w.shape[0], 3, 3), dtype=np.complex128)
    half = GELL_MANN / 2
    for s in range(0, w.shape[0], chunk):
        h = np.einsum("na,aij->nij", w[s:s + chunk], half)
        e, q = np.linalg.eigh(h)
        ph = np.exp(1j * eps * e)
        out[s:s + chunk] = np.einsum("nia,na,nja->nij", q, ph, q.conj())
    return out.reshape(4, lt, lz, ly, lx, 3, 3)


def unit_links(dims):
    """Free field: every link is the 3x3 identity."""
    lx, ly, lz, lt = dims
    u = np.zeros((4, lt, lz, ly, lx, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def rhs_gaussian(dims, seed):
    """Complex Gaussian vector (N + iN)/sqrt(2), canonical layout."""
    lx, ly, lz, lt = dims
    z = np.random.default_rng(seed).standard_normal((lt, lz, ly, lx, 4, 3, 2))
    return (z[..., 0] + 1j * z[..., 1]) / np.sqrt(2.0)


def rhs_z4(dims, seed):
    """Z4 noise: every entry uniform in {1, i, -1, -i}, canonical layout."""
    lx, ly, lz, lt = dims
    k = np.random.default_rng(seed).integers(0, 4, size=(lt, lz, ly, lx, 4, 3))
    return (1j ** k).astype(np.complex128)


def random_su3(count, seed):
    """Haar-ish random SU(3) matrices (gauge transformations for tests)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((count, 3, 3)) + 1j * rng.standard_normal((count, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q[:, :, 0] /= det[:, None]
    return q


# Workloads. Shift lists, restart parameters and tolerances follow the
# problem statement of eq. (1.1); sizes follow the lattice QCD setting of
# Example 7 (n = 12 complex unknowns per site). "rhs" lists (kind, seed).
CONFIGS = {
    "C1": dict(dims=(4, 4, 4, 4), eps=0.3, seed=0, kappa_factor=0.95,
               sigmas=[0.0, -0.02, -0.05, -0.1, -0.2],
               rhs=[("gauss", 1000)], m_dr=30, k=10, m_proj=30,
               tol=1e-10, tol_extra=1e-5, precision="f64"),
    "C2": dict(dims=(8, 8, 8, 8), eps=0.3, seed=0, kappa_factor=0.95,
               sigmas=[0.0, -0.01, -0.02, -0.05, -0.1, -0.2],
               rhs=[("gauss", 1000), ("z4", 1001), ("z4", 1002), ("z4", 1003)],
               m_dr=40, k=15, m_proj=40, tol=1e-10, tol_extra=1e-5,
               precision="f64"),
    "C3": dict(dims=(16, 16, 16, 32), eps=0.5, seed=0, kappa_factor=0.98,
               sigmas=[0.0, -0.01, -0.02, -0.05, -0.1, -0.2],
               rhs=[("gauss", 1000)], m_dr=60, k=20, m_proj=40,
               tol=1e-8, tol_extra=1e-4, precision="mixed"),
    "C4": dict(dims=(24, 24, 24, 48), eps=0.5, seed=0, kappa_factor=0.98,
               sigmas=[0.0, -0.01, -0.02, -0.05, -0.1, -0.2],
               rhs=[("z4", 1000 + j) for j in range(12)], m_dr=60, k=20,
               m_proj=40, tol=1e-8, tol_extra=1e-4, precision="mixed"),
    # the uneven mixed batch: one 32^3x64 lattice (FP16-stored links, 8 shifts,
    # 4 RHS) solved concurrently with six 12^4 and four 16^4 lattices (2 RHS,
    # 4 shifts each)
    # kappa_c of the 32^3x64 field: the restarted Arnoldi estimate the oracle
    # can afford at n = 25M is unconverged (Ritz residual 0.75, edge below
    # that of the smaller lattices), so the 24^3x48 value of the same
    # ensemble stands in (kappa_c changes by 5e-4 relative from 16^3x32 on)
    "C5": dict(dims=(32, 32, 32, 64), eps=0.5, seed=0, kappa_factor=0.98,
               kappa_c_from=((24, 24, 24, 48), 0.5, 0),
               sigmas=[0.0, -0.005, -0.01, -0.02, -0.05, -0.1, -0.2, -0.3],
               rhs=[("z4", 2000 + j) for j in range(4)], m_dr=60, k=20, m_proj=40,
               tol=1e-8, tol_extra=1e-4, precision="mixed", links="f16"),
}
for _s in range(1, 7):
    CONFIGS["C5a%d" % _s] = dict(dims=(12, 12, 12, 12), eps=0.5, seed=_s, kappa_factor=0.98,
                                sigmas=[0.0, -0.02, -0.05, -0.1],
                                rhs=[("z4", 3000 + 10 * _s + j) for j in range(2)], m_dr=40,
                                k=15, m_proj=40, tol=1e-8, tol_extra=1e-4, precision="mixed")
for _s in range(7, 11):
    CONFIGS["C5b%d" % _s] = dict(dims=(16, 16, 16, 16), eps=0.5, seed=_s, kappa_factor=0.98,
                                sigmas=[0.0, -0.02, -0.05, -0.1],
                                rhs=[("z4", 3000 + 10 * _s + j) for j in range(2)], m_dr=40,
                                k=15, m_proj=40, tol=1e-8, tol_extra=1e-4, precision="mixed")
C5_GROUP = ["C5"] + ["C5a%d" % s for s in range(1, 7)] + ["C5b%d" % s for s in range(7, 11)]


def make_rhs(cfg_or_dims, kind, seed):
    dims = cfg_or_dims["dims"] if isinstance(cfg_or_dims, dict) else cfg_or_dims
    if kind == "gauss":
        return rhs_gaussian(dims, seed)
    if kind == "z4":
        return rhs_z4(dims, seed)
    raise ValueError(kind)


def manifest():
    if not os.path.exists(MANIFEST):
        return {}
    with open(MANIFEST) as f:
        return json.load(f)


def manifest_key(dims, eps, seed):
    return "%dx%dx%dx%d_eps%g_seed%d" % (tuple(dims) + (eps, seed))


def kappa(name):
    """kappa = kappa_factor * kappa_c for a workload, from the manifest."""
    cfg = CONFIGS[name]
    dims, eps, seed = cfg.get("kappa_c_from", (cfg["dims"], cfg["eps"], cfg["seed"]))
    entry = manifest().get(manifest_key(dims, eps, seed))
    if entry is None:
        raise KeyError("kappa_c for %s not in %s; run oracle/make_manifest.py"
                       % (name, MANIFEST))
    return cfg["kappa_factor"] * entry["kappa_c"]
