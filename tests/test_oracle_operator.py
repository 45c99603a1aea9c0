"""Pins of the oracle's lattice tables, gauge field and Wilson operator
against facts fixed by the mathematics (not by re-running the oracle)."""
import numpy as np
import pytest

import synth
from oracle import kappa, lattice, wilson


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 6, 4), (4, 4, 4, 8)])
def test_tables_invariants(dims):
    eo, nbr, sign = lattice.tables(dims)
    vol = int(np.prod(dims))
    # bijection lex -> eo
    assert sorted(eo.tolist()) == list(range(vol))
    # neighbour of neighbour in the opposite direction is the site itself
    for mu in range(4):
        assert np.array_equal(nbr[nbr[:, mu], mu + 4], np.arange(vol))
        assert np.array_equal(nbr[nbr[:, mu + 4], mu], np.arange(vol))
    # every hop flips parity: parity of eo position p*V/2+... is eo >= V/2
    par = (np.arange(vol) >= vol // 2).astype(int)
    for d in range(8):
        assert np.all(par[nbr[:, d]] == 1 - par)
    # t-boundary signs: V/Lt sites leave forward and V/Lt backward
    assert int((sign == -1).sum()) == 2 * vol // dims[3]
    assert np.all(sign[:, :3] == 1) and np.all(sign[:, 4:7] == 1)


def test_tables_small_explicit():
    # 2x2x2x2: site (1,0,0,0) has lex 1, parity 1, eo = 8 + 0 = 8
    eo, nbr, sign = lattice.tables((2, 2, 2, 2))
    assert eo[0] == 0 and eo[1] == 8 and eo[2] == 9 and eo[3] == 1
    # +x neighbour of the origin is (1,0,0,0) -> eo 8; -t of origin crosses
    assert nbr[0, 0] == 8
    assert sign[0, 7] == -1 and sign[0, 3] == 1


def test_links_special_unitary():
    u = synth.gauge_links((4, 4, 2, 2), 0.5, 3).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.abs(np.einsum("nab,ncb->nac", u, u.conj()) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14


def test_gamma_algebra():
    g = wilson.GAMMA
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * (a == b) * np.eye(4), atol=0)
        assert np.linalg.matrix_rank(np.eye(4) - g[a]) == 2
    assert np.allclose(wilson.GAMMA5, np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (2, 2, 2, 4), (4, 2, 2, 4)])
def test_free_field_spectrum(dims):
    """Unit links: dense spectrum equals the Fourier closed form."""
    D = wilson.dense_hop(synth.unit_links(dims))
    ev = np.linalg.eigvals(D)
    ex = wilson.free_field_eigenvalues(dims)
    key = lambda z: np.lexsort((np.round(z.imag, 8), np.round(z.real, 8)))
    a = ev[key(ev)]
    b = ex[key(ex)]
    assert np.abs(a - b).max() < 1e-12


def test_dense_assembly_matches_definition():
    u = synth.gauge_links((2, 2, 2, 2), 0.3, 0)
    a = wilson.dense_hop(u)
    b = wilson.dense_hop_from_definition(u)
    assert np.abs(a - b).max() < 1e-14
    # periodic in every direction too
    a = wilson.dense_hop(u, (1, 1, 1, 1))
    b = wilson.dense_hop_from_definition(u, (1, 1, 1, 1))
    assert np.abs(a - b).max() < 1e-14


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 4)
    u = synth.gauge_links(dims, 0.3, 1)
    op = wilson.WilsonOperator(u, 0.13)
    x = synth.rhs_gaussian(dims, 5).ravel()
    y = synth.rhs_gaussian(dims, 6).ravel()
    g5 = lambda v: wilson.gamma5_flat(v, op.shape)
    lhs = np.vdot(y, g5(op(g5(x))))
    rhs = np.vdot(op(y), x)
    assert abs(lhs - rhs) <= 1e-13 * abs(rhs)


def test_gauge_covariance():
    dims = (4, 4, 2, 4)
    lx, ly, lz, lt = dims
    u = synth.gauge_links(dims, 0.5, 2)
    om = synth.random_su3(lx * ly * lz * lt, 9).reshape(lt, lz, ly, lx, 3, 3)
    up = np.empty_like(u)
    for mu in range(4):
        om_fwd = np.roll(om, -1, axis=3 - mu)     # Omega(x + mu), periodic
        up[mu] = np.einsum("tzyxab,tzyxbc,tzyxdc->tzyxad", om, u[mu], om_fwd.conj())
    psi = synth.rhs_gaussian(dims, 4)
    rot = lambda p: np.einsum("tzyxab,tzyxsb->tzyxsa", om, p)
    lhs = wilson.hop(up, rot(psi))
    rhs = rot(wilson.hop(u, psi))
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(rhs).max()


def test_kappa_c_free_field():
    for lt in (4, 8):
        dims = (2, 2, 2, lt)
        ev = kappa.rightmost_dense(synth.unit_links(dims))
        kc = kappa.kappa_c_from_eigs(ev)
        assert abs(kc - 1 / (6 + 2 * np.cos(np.pi / lt))) < 1e-12
        assert abs(kappa.bisect_kappa_c(ev) - kc) < 1e-9 * kc
    assert abs(1 / (6 + 2 * np.cos(np.pi / 4)) - 0.134876) < 1e-6


def test_kappa_c_arpack_matches_dense():
    u = synth.gauge_links((2, 2, 4, 4), 0.3, 0)
    kd = kappa.kappa_c_from_eigs(kappa.rightmost_dense(u))
    ka = kappa.kappa_c_from_eigs(kappa.rightmost_arpack(u, ncv=40))
    assert abs(kd - ka) < 1e-9 * kd


def test_kappa_c_restarted_arnoldi_matches_dense():
    """The large-lattice estimate (restarted Arnoldi on D) agrees with the
    dense spectrum's rightmost eigenvalue."""
    u = synth.gauge_links((2, 4, 2, 4), 0.5, 1)
    kd = kappa.kappa_c_from_eigs(kappa.rightmost_dense(u))
    ev, res = kappa.rightmost_restarted_arnoldi(u, m=40, restarts=6)
    ka = kappa.kappa_c_from_eigs(ev)
    assert abs(ka - kd) <= 2e-3 * kd
