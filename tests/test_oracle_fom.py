"""Pins of the oracle's FOM-Sh / FOM-DR-Sh (Sec. 3, Examples 2 and 3), the
Galerkin comparison method: the Galerkin condition against a Krylov basis
built independently (power basis + QR), parallel residuals, the classical
identity between FOM and GMRES residual norms of one cycle, exactness when
the Krylov space fills the whole space, and the paper's statements on the
bidiagonal matrix of Example 1."""
import json
import os

import numpy as np

from oracle import gmres

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
norm = np.linalg.norm


def dense(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    A += shift * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return A, b


def example1():
    d = np.concatenate([[0.1], np.arange(1, 1000)]).astype(np.complex128)

    def mv(v):
        w = d * v
        w[:-1] += v[1:]
        return w
    return mv


def one_cycle(A, b, sig, m, fom):
    return gmres.gmres_dr_sh(lambda v: A @ v, b, sig, m, 0, 0.0, max_cycles=1, fom=fom)


def test_galerkin_condition_and_parallel_residuals():
    A, b = dense(30, 1)
    sig = [0.5, -0.3 + 0.2j, 1.1]
    m = 6
    r = one_cycle(A, b, sig, m, True)
    K = np.stack([np.linalg.matrix_power(A, j) @ b for j in range(m)], axis=1)
    Q, _ = np.linalg.qr(K)
    res = [b - (A - s * np.eye(30)) @ r["x"][i] for i, s in enumerate(sig)]
    for i in range(len(sig)):
        assert norm(Q.conj().T @ res[i]) <= 1e-10 * norm(res[i])
        cosang = abs(np.vdot(res[0], res[i])) / (norm(res[0]) * norm(res[i]))
        assert abs(cosang - 1) <= 1e-10
        assert abs(norm(res[i]) / norm(b) - r["history"][-1]["res"][i]) <= 1e-10 * norm(res[i]) / norm(b)
    # GMRES-Sh's base system is not Galerkin: its residual is not orthogonal
    g = one_cycle(A, b, sig, m, False)
    rg = b - (A - sig[0] * np.eye(30)) @ g["x"][0]
    assert norm(Q.conj().T @ rg) > 1e-3 * norm(rg)


def test_fom_gmres_residual_identity():
    """One cycle from the same start: ||r_F(m)|| = ||r_G(m)|| /
    sqrt(1 - (||r_G(m)|| / ||r_G(m-1)||)^2) (base shift)."""
    A, b = dense(40, 2, shift=1.5)
    sig = [0.2 + 0.1j]
    for m in (3, 5, 8):
        f = one_cycle(A, b, sig, m, True)["history"][-1]["r1"]
        g = one_cycle(A, b, sig, m, False)["history"][-1]["r1"]
        g1 = one_cycle(A, b, sig, m - 1, False)["history"][-1]["r1"]
        want = g / np.sqrt(1 - (g / g1) ** 2)
        assert abs(f - want) <= 1e-9 * want, (m, f, want)


def test_exact_when_krylov_space_is_full():
    A, b = dense(12, 3)
    sig = [0.0, 0.7, -0.4 + 0.3j]
    r = gmres.gmres_dr_sh(lambda v: A @ v, b, sig, 12, 0, 1e-12, max_cycles=1, fom=True)
    for i, s in enumerate(sig):
        x = np.linalg.solve(A - s * np.eye(12), b)
        assert norm(r["x"][i] - x) <= 1e-9 * norm(x)


def test_fomdr_restart_keeps_ritz_pairs():
    """After a FOM-DR restart the new H_bar_k satisfies A V_k = V_{k+1} H_bar_k
    with V_{k+1} orthonormal, and its square part has the kept Ritz values
    (plus sigma_1) as eigenvalues."""
    A, b = dense(60, 4, shift=1.5)
    sig = [0.3, 0.0]
    r = gmres.gmres_dr_sh(lambda v: A @ v, b, sig, 15, 4, 1e-6, max_cycles=40, fom=True)
    assert r["converged"] and r["defl"] is not None
    V, Hk = r["defl"]
    k = Hk.shape[1]
    assert norm(V.conj().T @ V - np.eye(k + 1)) <= 1e-10
    assert norm(A @ V[:, :k] - V @ Hk) <= 1e-9 * norm(Hk)
    ev = np.sort_complex(np.linalg.eigvals(Hk[:k, :]))
    th = np.sort_complex(r["history"][-1]["theta"] + sig[0])
    assert np.abs(ev - th).max() <= 1e-8 * np.abs(th).max()


def test_example2_statements():
    """FOM(40)-Sh, shifts 0.4, 0, -1: sigma = -1 drops below 1e-8 within 400
    iterations, which GMRES(40)-Sh does not reach; for the base shift 0.4
    GMRES is the better of the two."""
    gold = GOLDEN["example2_fom_sigma_m1"]
    mv = example1()
    b = np.random.default_rng(0).standard_normal(1000) + 0j
    sig = [0.4, 0, -1]
    cyc = gold["iterations"] // 40
    f = gmres.gmres_dr_sh(mv, b, sig, 40, 0, gold["tol"], max_cycles=cyc, fom=True)
    g = gmres.gmres_dr_sh(mv, b, sig, 40, 0, gold["tol"], max_cycles=cyc)
    fr = np.array([h["res"] for h in f["history"]])
    gr = np.array([h["res"] for h in g["history"]])
    assert f["mvps"] <= gold["iterations"]
    assert fr[:, 2].min() <= gold["tol"]
    assert gr[:, 2].min() > gold["tol"]
    assert gr[-1, 0] < fr[-1, 0]
    for i, s in enumerate(sig):   # the tracked residuals are the true ones
        t = norm(gmres.true_residual(mv, b, f["x"][i], s)) / norm(b)
        assert abs(t - fr[-1, i]) <= 1e-6 * t + 1e-14


def test_example3_fomdr_removes_two_eigenvalues():
    """Base shift 0, second shift 1.4, cycle length 80: FOM-Sh stays far from
    convergence on the 1.4 system, GMRES-Sh does better, and FOM-DR-Sh(80,2)
    converges; its two Ritz values are the matrix's smallest eigenvalues
    0.1 and 1."""
    gold = GOLDEN["example3_fomdr"]
    mv = example1()
    b = np.random.default_rng(0).standard_normal(1000) + 0j
    sig, m, k = gold["shifts"], gold["m"], gold["k"]
    fd = gmres.gmres_dr_sh(mv, b, sig, m, k, 1e-8, max_cycles=6, fom=True)
    assert fd["converged"]
    th = np.sort(fd["history"][-1]["theta"].real)
    assert np.abs(th - [0.1, 1.0]).max() <= 1e-6
    f = gmres.gmres_dr_sh(mv, b, sig, m, 0, 1e-8, max_cycles=6, fom=True)
    g = gmres.gmres_dr_sh(mv, b, sig, m, 0, 1e-8, max_cycles=6)
    fr = f["history"][-1]["res"][1]
    gr = g["history"][-1]["res"][1]
    assert fr > 1e-3
    assert gr < fr
