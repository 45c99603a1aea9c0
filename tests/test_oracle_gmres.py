"""Pins of the oracle's Krylov solvers against the mathematics and against
numbers the paper prints. None of these re-run the oracle's own formulas as
the check: they use dense LU, brute-force least squares, SciPy's GMRES,
exact invariants of the recurrences and the paper's example results."""
import numpy as np
import pytest
import scipy.linalg as sl
import scipy.sparse.linalg as sla

import json
import os

import synth
from oracle import gmres, wilson

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
norm = np.linalg.norm


def cond1(M):
    """1-norm condition number estimate (LAPACK gecon on an LU factor)."""
    lu, piv = sl.lu_factor(M)
    rcond, info = sl.lapack.zgecon(lu, np.linalg.norm(M, 1), norm="1")
    return 1.0 / rcond


# --------------------------------------------------------------------------
# operators
# --------------------------------------------------------------------------
def bidiag_matvec():
    """Example 1's matrix: n=1000, diagonal 0.1, 1, 2, ..., 999, superdiagonal 1."""
    d = np.concatenate([[0.1], np.arange(1, 1000)]).astype(np.complex128)

    def mv(v):
        w = d * v
        w[:-1] += v[1:]
        return w
    return mv, d


def bidiag_dense():
    _, d = bidiag_matvec()
    return np.diag(d) + np.diag(np.ones(999), 1)


@pytest.fixture(scope="module")
def wil():
    """C1's operator: 4^4, eps 0.3, seed 0, kappa = 0.95 kappa_c."""
    cfg = synth.CONFIGS["C1"]
    u = synth.gauge_links(cfg["dims"], cfg["eps"], cfg["seed"])
    op = wilson.WilsonOperator(u, synth.kappa("C1"))
    b = synth.rhs_gaussian(cfg["dims"], 1000).ravel()
    return op, b, cfg


@pytest.fixture(scope="module")
def wil_dense(wil):
    op, b, cfg = wil
    return np.eye(op.n) - op.kappa * wilson.dense_hop(op.links, op.bc)


# --------------------------------------------------------------------------
# Arnoldi (eq. 2.2) and the base minimum-residual property (Sec. 2.1)
# --------------------------------------------------------------------------
def test_arnoldi_recurrence_and_orthonormality(wil):
    op, b, _ = wil
    m = 25
    V = np.zeros((op.n, m + 1), complex)
    H = np.zeros((m + 1, m), complex)
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(m):
        assert not gmres.arnoldi_step(op, V, H, j)
    AV = np.stack([op(V[:, j]) for j in range(m)], axis=1)
    assert np.linalg.norm(AV - V @ H) <= 1e-13 * np.linalg.norm(H)
    assert np.abs(V.conj().T @ V - np.eye(m + 1)).max() <= 1e-13
    assert np.allclose(np.tril(H, -2), 0)


def test_base_min_residual_brute_force(wil):
    """d_1 of the first cycle equals lstsq over W = (A - sigma_1) V_m formed
    with m explicit extra products."""
    op, b, cfg = wil
    sig = np.array(cfg["sigmas"], complex)
    m = 20
    out = gmres.gmres_dr_sh(op, b, sig, m, 5, 1e-30, max_cycles=1)
    V = np.zeros((op.n, m + 1), complex)
    H = np.zeros((m + 1, m), complex)
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(m):
        gmres.arnoldi_step(op, V, H, j)
    W = np.stack([op.shifted(V[:, j], sig[0]) for j in range(m)], axis=1)
    d = np.linalg.lstsq(W, b, rcond=None)[0]
    x1 = V[:, :m] @ d
    assert np.linalg.norm(out["x"][0] - x1) <= 1e-10 * np.linalg.norm(x1)
    r_true = np.linalg.norm(b - W @ d) / np.linalg.norm(b)
    assert abs(out["history"][0]["r1"] - r_true) <= 1e-10 * r_true


# --------------------------------------------------------------------------
# GMRES-DR-Sh (Sec. 3)
# --------------------------------------------------------------------------
def test_dr_sh_solutions_match_dense_lu(wil, wil_dense):
    op, b, cfg = wil
    sig = np.array(cfg["sigmas"], complex)
    out = gmres.gmres_dr_sh(op, b, sig, cfg["m_dr"], cfg["k"], cfg["tol"])
    assert out["converged"]
    # structure of the cost: m products in the first cycle, m-k after
    assert out["mvps"] == cfg["m_dr"] + (out["cycles"] - 1) * (cfg["m_dr"] - cfg["k"])
    for i, s in enumerate(sig):
        M = wil_dense - s * np.eye(op.n)
        xs = np.linalg.solve(M, b)
        cond = cond1(M)
        err = np.linalg.norm(out["x"][i] - xs) / np.linalg.norm(xs)
        assert err <= cond * cfg["tol"]
        r = np.linalg.norm(b - M @ out["x"][i]) / np.linalg.norm(b)
        assert r <= 2 * cfg["tol"]


@pytest.mark.parametrize("cycles", [1, 2, 4])
def test_dr_sh_residuals_collinear(wil, cycles):
    """After each cycle r_i = beta_i r_1 for the true residuals."""
    op, b, cfg = wil
    sig = np.array(cfg["sigmas"], complex)
    out = gmres.gmres_dr_sh(op, b, sig, 20, 6, 1e-30, max_cycles=cycles)
    r1 = gmres.true_residual(op, b, out["x"][0], sig[0])
    for i in range(1, len(sig)):
        ri = gmres.true_residual(op, b, out["x"][i], sig[i])
        assert np.linalg.norm(ri - out["beta"][i] * r1) <= 1e-12 * np.linalg.norm(b)
    # the shortcut norm (2.6) is the true norm
    assert abs(np.linalg.norm(r1) / np.linalg.norm(b) - out["history"][-1]["r1"]) <= 1e-12


def test_dr_restart_keeps_eigen_recurrence(wil):
    """A V_k = V_{k+1} H_bar_k holds for the compressed basis (eq. 2.9), and
    the harmonic Ritz residuals are all parallel to the GMRES residual s."""
    op, b, cfg = wil
    out = gmres.gmres_dr_sh(op, b, [0.0], 30, 10, 1e-8)
    m, k = 30, 10
    V = np.zeros((op.n, m + 1), complex)
    H = np.zeros((m + 1, m), complex)
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(m):
        gmres.arnoldi_step(op, V, H, j)
    c = np.zeros(m + 1, complex)
    c[0] = np.linalg.norm(b)
    d = np.linalg.lstsq(H, c, rcond=None)[0]
    s = c - H @ d
    theta, g = gmres.harmonic_ritz(H, 0.0)
    for t, gv in zip(theta, g.T):
        res = H @ gv - t * np.concatenate([gv, [0]])
        # parallel to s: the component orthogonal to s vanishes
        res_perp = res - s * (np.vdot(s, res) / np.vdot(s, s))
        assert np.linalg.norm(res_perp) <= 1e-9 * max(np.linalg.norm(res), 1e-12) + 1e-12
    Vk1, Hk, cn, _ = gmres.dr_restart(V, H, s, 0.0, k)
    AVk = np.stack([op(Vk1[:, j]) for j in range(k)], axis=1)
    assert np.linalg.norm(AVk - Vk1 @ Hk) <= 1e-12 * np.linalg.norm(Hk)
    # the residual stays in the new space: V_{m+1} s = V_{k+1} c_new
    assert np.linalg.norm(V @ s - Vk1 @ cn) <= 1e-12 * np.linalg.norm(s)
    # the exported pair of a run satisfies the same recurrence
    Vk1, Hk = out["defl"]
    AVk = np.stack([op(Vk1[:, j]) for j in range(k)], axis=1)
    assert np.linalg.norm(AVk - Vk1 @ Hk) <= 1e-11 * np.linalg.norm(Hk)


def test_dr_subspace_is_augmented_krylov(wil):
    """Eq. (2.7): after a restart, span V_m = span{y_1..y_k, r0, A r0, ...,
    A^{m-k-1} r0} with y the harmonic Ritz vectors (principal angles)."""
    op, b, _ = wil
    m, k = 16, 5
    V = np.zeros((op.n, m + 1), complex)
    H = np.zeros((m + 1, m), complex)
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(m):
        gmres.arnoldi_step(op, V, H, j)
    c = np.zeros(m + 1, complex)
    c[0] = np.linalg.norm(b)
    d = np.linalg.lstsq(H, c, rcond=None)[0]
    s = c - H @ d
    theta, g = gmres.harmonic_ritz(H, 0.0)
    sel = gmres.select_smallest(theta, k)
    Y = V[:, :m] @ g[:, sel]
    r0 = V @ s
    Vk1, Hk, cn, _ = gmres.dr_restart(V, H, s, 0.0, k)
    V2 = np.zeros_like(V)
    H2 = np.zeros_like(H)
    V2[:, :k + 1] = Vk1
    H2[:k + 1, :k] = Hk
    for j in range(k, m):
        gmres.arnoldi_step(op, V2, H2, j)
    kry = [r0]
    for _ in range(m - k - 1):
        kry.append(op(kry[-1]))
    S = np.column_stack([Y] + kry)
    Qs, _ = np.linalg.qr(S)
    ang = sl.subspace_angles(Qs, V2[:, :m])
    assert np.max(ang) <= 1e-7


def test_k0_single_shift_is_textbook_gmres():
    """k = 0, one shift: GMRES(m). Per-cycle iterates match SciPy's."""
    mv, _ = bidiag_matvec()
    A = bidiag_dense()
    b = np.random.default_rng(3).standard_normal(1000) + 0j
    m = 15
    out_hist = []
    for c in range(1, 6):
        o = gmres.gmres_dr_sh(mv, b, [0.0], m, 0, 1e-30, max_cycles=c)
        out_hist.append(o["x"][0])
    xs = []
    sla.gmres(A, b, restart=m, maxiter=5, rtol=1e-30, atol=0,
              callback=lambda x: xs.append(x.copy()), callback_type="x")
    for a, s in zip(out_hist, xs):
        assert np.linalg.norm(a - s) <= 1e-9 * np.linalg.norm(s)


def test_duplicate_shift(wil):
    op, b, _ = wil
    out = gmres.gmres_dr_sh(op, b, [0.0, 0.0], 20, 5, 1e-8)
    assert np.linalg.norm(out["x"][1] - out["x"][0]) <= 1e-12 * np.linalg.norm(out["x"][0])
    assert abs(out["beta"][1] - 1) <= 1e-12


def test_lucky_breakdown_plane_wave():
    """Free field, b = plane wave: the Krylov space has dimension <= 4, the
    cycle truncates and every shift is solved exactly."""
    dims = (4, 4, 4, 4)
    op = wilson.WilsonOperator(synth.unit_links(dims), 0.1)
    lt, lz, ly, lx = 4, 4, 4, 4
    t, z, y, x = np.meshgrid(range(lt), range(lz), range(ly), range(lx), indexing="ij")
    ph = np.exp(1j * (2 * np.pi * (x + 2 * y) / 4 + np.pi * 3 * t / 4))
    chi = np.zeros((4, 3), complex)
    chi[0, 1] = 1
    chi[2, 1] = 0.5j
    b = (ph[..., None, None] * chi).ravel()
    sig = [0.0, -0.3]
    out = gmres.gmres_dr_sh(op, b, sig, 10, 3, 1e-12)
    assert out["mvps"] <= 4 and out["cycles"] == 1
    for i, s in enumerate(sig):
        r = gmres.true_residual(op, b, out["x"][i], s)
        assert np.linalg.norm(r) <= 1e-13 * np.linalg.norm(b)


def test_paper_example4_mvp_count():
    """Example 4 / Example 1: GMRES-DR(25,10)-Sh on the bidiagonal matrix,
    sigma = 0, -0.4, -2, reaches relative residual 1e-10 in 250 matrix-
    vector products (25 + 15 c with c = 15). Random b: allow one cycle."""
    mv, _ = bidiag_matvec()
    counts = []
    for seed in range(5):
        b = np.random.default_rng(seed).standard_normal(1000) + 0j
        o = gmres.gmres_dr_sh(mv, b, [0, -0.4, -2], 25, 10, 1e-10)
        assert o["converged"]
        assert (o["mvps"] - 25) % 15 == 0
        counts.append(o["mvps"])
    want = GOLDEN["example4_mvps_to_1e-10"]["value"]
    assert np.median(counts) == want
    assert all(abs(c - want) <= 15 for c in counts)


# --------------------------------------------------------------------------
# GMRES-Proj-Sh, extra right-hand side and correction (Sec. 4)
# --------------------------------------------------------------------------
def test_theorem1_exact_eigenvectors_keep_residuals_parallel(wil_dense):
    """Theorem 1: minres projection over exact eigenvectors keeps
    r_i = beta_i r_1 (here with dense eigenvectors of a 2^4 operator)."""
    u = synth.gauge_links((2, 2, 2, 2), 0.3, 0)
    A = np.eye(192) - 0.12 * wilson.dense_hop(u)
    lam, Z = np.linalg.eig(A)
    Z = Z[:, np.argsort(np.abs(lam))[:6]]
    rng = np.random.default_rng(1)
    r0 = rng.standard_normal(192) + 1j * rng.standard_normal(192)
    sig = [0.0, -0.1, -0.3]
    beta = [1.0, 0.7 - 0.2j, 1.3]
    res = []
    for s, bt in zip(sig, beta):
        W = (A - s * np.eye(192)) @ Z
        d = np.linalg.lstsq(W, bt * r0, rcond=None)[0]
        res.append(bt * r0 - W @ d)
    for i in (1, 2):
        assert np.linalg.norm(res[i] - beta[i] * res[0]) <= 1e-12 * np.linalg.norm(r0)


def _defl_for_bidiag(tol=1e-10):
    mv, _ = bidiag_matvec()
    b1 = np.random.default_rng(100).standard_normal(1000) + 0j
    o = gmres.gmres_dr_sh(mv, b1, [0, -2], 25, 10, tol)
    return mv, o["defl"]


@pytest.mark.parametrize("cycles", [1, 2, 3])
def test_proj_sh_vk1_invariant(cycles):
    """Eq. (4.1): after every projection + GMRES-Sh cycle the true residuals
    satisfy r_i = beta_i r_1 + Gamma_i v_{k+1}."""
    mv, defl = _defl_for_bidiag()
    sig = np.array([0, -0.4, -2], complex)
    b = np.random.default_rng(7).standard_normal(1000) + 0j
    o = gmres.gmres_proj_sh(mv, b, sig, defl, 15, 1e-30, max_cycles=cycles)
    r1 = gmres.true_residual(mv, b, o["x"][0], sig[0])
    assert np.linalg.norm(r1 - o["r1"]) <= 1e-11 * np.linalg.norm(b)
    v = defl[0][:, -1]
    for i in (1, 2):
        ri = gmres.true_residual(mv, b, o["x"][i], sig[i])
        pred = o["beta"][i] * r1 + o["gam"][i] * v
        assert np.linalg.norm(ri - pred) <= 1e-11 * np.linalg.norm(b)
    assert abs(o["gam"][1]) > 1e-8   # the tracked component is really there


def test_extra_rhs_and_correction_reach_tolerance():
    """Example 5/6 setting: after the correction every shift meets the
    tolerance (relative), while before it the non-base residual plateaus
    far above it (Example 5: about 4e-3)."""
    mv, _ = bidiag_matvec()
    rng = np.random.default_rng(11)
    B = rng.standard_normal((2, 1000)) + 0j
    sig = np.array([0, -2], complex)
    tol = 1e-8
    o = gmres.solve_all(mv, B, sig, 25, 10, 15, tol, 1e-4)
    assert np.all(o["resid"][0] <= 2 * tol)
    assert np.all(o["resid"][1] <= 10 * tol)
    # uncorrected run: same projection + cycles, no correction
    first = gmres.gmres_dr_sh(mv, B[0], sig, 25, 10, tol)
    pr = gmres.gmres_proj_sh(mv, B[1], sig, first["defl"], 15, tol)
    unc = np.linalg.norm(gmres.true_residual(mv, B[1], pr["x"][1], sig[1])) / np.linalg.norm(B[1])
    assert unc > 100 * tol
    # Example 5's plateau is printed as about 4e-3 (rtol 1e-6); same order here
    plateau = GOLDEN["example5_uncorrected_plateau"]["value"]
    pr6 = gmres.gmres_proj_sh(mv, B[1], sig, gmres.gmres_dr_sh(mv, B[0], sig, 25, 10, 1e-6)["defl"], 15, 1e-6)
    unc6 = np.linalg.norm(gmres.true_residual(mv, B[1], pr6["x"][1], sig[1]))
    assert plateau / 10 <= unc6 <= plateau * 30
    # the extra system: (A - sigma_i) s_i = v_{k+1} to about tol_extra
    v = o["defl"][0][:, -1]
    r = gmres.true_residual(mv, v, o["extra"]["s"][1], sig[1])
    assert np.linalg.norm(r) <= 1e-3


def test_table42_trend():
    """Table 4.2: accuracy after correction degrades as the extra-RHS
    tolerance loosens, and with tol_extra = 1e-6 it is close to the desired
    tolerance (absolute ||r||, ||b|| about sqrt(1000))."""
    mv, _ = bidiag_matvec()
    rng = np.random.default_rng(0)
    B = rng.standard_normal((2, 1000)) + 0j
    sig = np.array([0, -2], complex)
    tol = 1e-8
    acc = []
    for te in (1e-6, 1e-4, 1e-2):
        o = gmres.solve_all(mv, B, sig, 25, 10, 15, tol, te)
        acc.append(o["resid"][1, 1] * np.linalg.norm(B[1]))
    assert acc[0] <= 10 * tol * np.linalg.norm(B[1])
    assert acc[0] <= acc[1] * 1.5 and acc[1] < acc[2]
    assert acc[2] > 10 * acc[0]
    # same order as the printed row for desired 1e-8: within 30x where the
    # extra system is solved tightly, 100x at tol_extra 1e-2 where the result
    # hinges on how far the last cycle overshoots (random b differs)
    row = GOLDEN["table42"]["rows"]["1e-8"]["after"]
    for got, te, band in zip(acc, (1e-6, 1e-4, 1e-2), (30, 30, 100)):
        want = row[GOLDEN["table42"]["tol_extra"].index(te)]
        assert want / band <= got <= want * band


def test_proj_sh_matches_dense(wil, wil_dense):
    """C1 operator, two RHS: every (shift, RHS) solution against dense LU."""
    op, b, cfg = wil
    sig = np.array(cfg["sigmas"], complex)
    B = np.stack([b, synth.rhs_z4(cfg["dims"], 1001).ravel()])
    o = gmres.solve_all(op, B, sig, 30, 10, 20, 1e-10, 1e-5)
    for j in range(2):
        for i, s in enumerate(sig):
            M = wil_dense - s * np.eye(op.n)
            xs = np.linalg.solve(M, B[j])
            err = np.linalg.norm(o["X"][j, i] - xs) / np.linalg.norm(xs)
            assert err <= cond1(M) * 1e-10
            assert o["resid"][j, i] <= 1e-9


def test_related_rhs_shift_independent():
    """Eq. (5.2): B^H B d = B^H b^j does not involve the shift, and every
    shifted residual after the projection is b^j - B d."""
    mv, _ = bidiag_matvec()
    A = bidiag_dense()
    rng = np.random.default_rng(5)
    b1 = rng.standard_normal(1000) + 0j
    B = np.stack([b1, b1 + 1e-4 * rng.standard_normal(1000)], axis=1)
    sig = [0.0, -0.4, -2.0]
    X = np.stack([np.linalg.solve(A - s * np.eye(1000), B) for s in sig])
    bj = b1 + 1e-4 * rng.standard_normal(1000)
    x0, r0 = gmres.related_rhs_start(B, X, bj)
    for i, s in enumerate(sig):
        ri = bj - (A - s * np.eye(1000)) @ x0[i]
        assert np.linalg.norm(ri - r0) <= 1e-8 * np.linalg.norm(bj)
    assert np.linalg.norm(r0) <= 1e-3 * np.linalg.norm(bj)

def test_table41_accurate_eigenvector_projection():
    """Table 4.1 (Example 4): after GMRES-DR(25,10)-Sh to 1e-10 on the first
    right-hand side, a second one by GMRES(15)-Proj-Sh projecting over only
    the leading k approximate eigenvectors. Per k, over three random right-
    hand side pairs: the median product count is within one cycle (15) of the
    paper's (one cycle of slack again for k = 2, where the printed 435 is
    two cycles above our 405), the worst non-base residual is within a factor
    30 of the printed level down to k = 6 (below that the paper's plateau is
    the tolerance reached), and fewer, more accurate vectors trade products
    for parallel residuals: products rise and the plateau falls as k drops."""
    mv, _ = bidiag_matvec()
    t = GOLDEN["table41"]
    sig = np.array([0, -0.4, -2], dtype=np.complex128)
    mv_k = {kp: [] for kp in t["k"]}
    res_k = {kp: [] for kp in t["k"]}
    for seed in range(3):
        b1 = np.random.default_rng(seed).standard_normal(1000) + 0j
        first = gmres.gmres_dr_sh(mv, b1, sig, 25, 10, 1e-10)
        assert first["converged"]
        b2 = np.random.default_rng(100 + seed).standard_normal(1000) + 0j
        for kp in t["k"]:
            o = gmres.gmres_proj_sh(mv, b2, sig, first["defl"], 15, 1e-10, 200, kp=kp)
            assert o["converged"]
            mv_k[kp].append(o["mvps"])
            res_k[kp].append(max(norm(gmres.true_residual(mv, b2, o["x"][i], sig[i])) / norm(b2)
                                 for i in (1, 2)))
    med_mv = [np.median(mv_k[kp]) for kp in t["k"]]
    med_res = [np.median(res_k[kp]) for kp in t["k"]]
    for want, got in zip(t["mvps"][:4], med_mv[:4]):
        assert abs(got - want) <= 15
    assert abs(med_mv[4] - t["mvps"][4]) <= 30
    for want, got in zip(t["lin_eqs_res"][:3], med_res[:3]):
        assert want / 30 <= got <= want * 30
    assert all(a <= b for a, b in zip(med_mv, med_mv[1:]))
    assert med_res[0] > med_res[2] > med_res[3]


def test_leading_projection_full_k_equals_standard():
    """With all k vectors the accurate-eigenvector projection is step 3-4 of
    GMRES-Proj-Sh (same solution updates and base residual); with exact
    eigenvectors (Theorem 1) the residuals of every shift stay parallel."""
    mv, d = bidiag_matvec()
    sig = np.array([0, -0.4, -2], dtype=np.complex128)
    b1 = np.random.default_rng(0).standard_normal(1000) + 0j
    Vk1, Hk = gmres.gmres_dr_sh(mv, b1, sig, 25, 10, 1e-10)["defl"]
    r = np.random.default_rng(1).standard_normal(1000) + 0j
    beta = np.array([1, 0.7 - 0.2j, 1.3 + 0.1j])
    xa = np.zeros((3, 1000), complex)
    xb = np.zeros((3, 1000), complex)
    ra = gmres.minres_projection_sh(Vk1, Hk, sig, xa, r.copy(), beta, np.zeros(3, complex))
    rb = gmres.leading_projection_sh(Vk1, Hk, sig, xb, r.copy(), beta, Hk.shape[1])
    assert np.abs(ra - rb).max() <= 1e-12 * norm(r)
    assert np.abs(xa - xb).max() <= 1e-12 * np.abs(xa).max()
    # exact eigenvectors: the bidiagonal matrix's 3 smallest, orthonormalised
    M = np.diag(d) + np.diag(np.ones(999), 1)
    lam, Z = np.linalg.eig(M)
    sel = np.argsort(np.abs(lam))[:3]
    Q, _ = np.linalg.qr(Z[:, sel])
    Vx = np.hstack([Q, np.zeros((1000, 1))])
    v = np.random.default_rng(2).standard_normal(1000) + 0j
    v -= Q @ (Q.conj().T @ v)
    Vx[:, 3] = v / norm(v)
    Hx = np.zeros((4, 3), complex)
    Hx[:3, :] = Q.conj().T @ M @ Q   # A Q = Q T, no v_{k+1} component
    x = np.zeros((3, 1000), complex)
    r0 = r.copy()
    r1 = gmres.leading_projection_sh(Vx, Hx, sig, x, r0, beta, 2)
    for i in range(1, 3):
        ri = beta[i] * r0 - (M @ x[i] - sig[i] * x[i])
        assert norm(ri - beta[i] * r1) <= 1e-10 * norm(r0)


def test_selection_order_and_conjugate_ties():
    """Harmonic Ritz selection: smallest |theta| first, ties by Re then Im;
    a conjugate pair whose computed moduli differ by rounding is a tie and
    its member with negative imaginary part comes first."""
    rng = np.random.default_rng(4)
    th = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    sel = gmres.select_smallest(th, 12)
    assert list(sel) == list(np.lexsort((th.imag, th.real, np.abs(th)))[:12])
    a = 3.0 + 0.25j
    pair = np.array([5.0, a * (1 + 3e-16), np.conj(a), 0.5, 7.0 + 1j])
    sel = gmres.select_smallest(pair, 3)
    assert list(sel) == [3, 2, 1]
