"""Deflated restarted GMRES for shifted systems with several right-hand sides.

Plain complex128 NumPy, one routine per step of the method, in the paper's
order and notation. ``matvec`` applies the unshifted A; shifts enter only
through H_bar - sigma I_bar (Sec. 2.1, shifted Arnoldi recurrence).

Readings of points the paper leaves open (all transposes are conjugate
transposes):

* Arnoldi uses classical Gram-Schmidt applied twice (CGS2). A lucky
  breakdown (||w|| <= 1e-14 ||A v_j||) truncates the cycle.
* The base least-squares problem is min ||c - (H_bar - sigma_1 I_bar) d||.
* The non-base shift solve (H_bar - sigma_i I_bar) d_i = beta_i c -
  beta_i^new s is taken as one square system [H_bar - sigma_i I_bar | s]
  [d_i; beta_i^new] = beta_i c. The paper solves it through a QR
  factorisation and its last row (Sec. 2.1); the two are the same system.
* GMRES-DR restart (Sec. 2.2; the restart details follow the cited GMRES-DR
  method): harmonic Ritz pairs of the base-shifted matrix, i.e. the
  eigenpairs of G = H_m + |h_{m+1,m}|^2 H_m^{-H} e_m e_m^H with
  H_m the leading m x m block of H_bar - sigma_1 I_bar; keep the k of
  smallest |theta| (ties: smaller Re, then smaller Im; moduli and real parts
  within 1e-10 relative are ties, so a conjugate pair of real data is split
  by the sign of Im, not by rounding); P_k = orthonormal
  basis of their eigenvectors padded with a zero row; p_{k+1} = s
  orthogonalised against P_k; H_bar_k <- P_{k+1}^H H_bar P_k (for A);
  V_{k+1} <- V_{m+1} P_{k+1}; c <- P_{k+1}^H s; v_{k+1} is
  re-orthogonalised against V_k.
* FOM-Sh / FOM-DR-Sh (Sec. 3, Examples 2 and 3): each shift takes the
  Galerkin solution (H_m - sigma_i I) y_i = beta_i c_{1:m}; the residuals are
  then all multiples of v_{m+1} and beta_i^new = (y_i)_m / (y_1)_m. FOM-DR
  deflates with Ritz pairs of H_m - sigma_1 I (smallest |theta|, same ties)
  and otherwise restarts exactly as GMRES-DR (the residual direction s is
  then e_{m+1}).
* Convergence is tested at the end of a cycle only, on
  max_i |beta_i| ||r_1|| / ||b|| (the shortcut norm of eq. (2.6)).
* After the last GMRES-DR-Sh cycle one more restart compression is made
  (no matrix-vector products) to hand (V_{k+1}, H_bar_k) to later
  right-hand sides.
* Correction phase (Sec. 4): gamma_i = v_{k+1}^H r_i with r_i the true
  residual of shift i.
"""
import numpy as np

BREAKDOWN_TOL = 1e-14


def norm(v):
    return float(np.linalg.norm(v))


def ibar(rows, cols):
    """The rows x cols identity I_bar of the shifted recurrence."""
    return np.eye(rows, cols, dtype=np.complex128)


# ----------------------------------------------------------------------------
# Arnoldi recurrence A V_m = V_{m+1} H_bar_m (eq. (2.2))
# ----------------------------------------------------------------------------
def arnoldi_step(matvec, V, H, j):
    """Extend the recurrence by column j: w = A v_j orthogonalised against
    v_0..v_j by CGS2. Returns True on a lucky breakdown."""
    w = matvec(V[:, j])
    w_norm0 = norm(w)
    Vj = V[:, :j + 1]
    h = Vj.conj().T @ w
    w = w - Vj @ h
    h2 = Vj.conj().T @ w
    w = w - Vj @ h2
    H[:j + 1, j] = h + h2
    hn = norm(w)
    H[j + 1, j] = hn
    if hn <= BREAKDOWN_TOL * w_norm0:
        H[j + 1, j] = 0.0
        return True
    V[:, j + 1] = w / hn
    return False


# ----------------------------------------------------------------------------
# GMRES-Sh small problems (Sec. 2.1; GMRES-DR-Sh steps 3-4)
# ----------------------------------------------------------------------------
def shifted_small_solves(H, c, sigmas, beta):
    """Base least squares and the collinear-residual solves for other shifts.

    H is (p+1) x p, c has p+1 entries. Returns (ds, s, beta_new) with ds[i]
    the update coefficients of shift i, s = c - (H - sigma_1 I_bar) d_1 and
    beta_new[i] such that r_i = beta_new[i] r_1 (beta_new[0] = 1).
    """
    p = H.shape[1]
    Ib = ibar(p + 1, p)
    Hs = H - sigmas[0] * Ib
    d1 = np.linalg.lstsq(Hs, c, rcond=None)[0]
    s = c - Hs @ d1
    ds = [d1]
    beta_new = np.ones(len(sigmas), dtype=np.complex128)
    exact = norm(s) <= BREAKDOWN_TOL * max(norm(c), 1e-300)
    for i in range(1, len(sigmas)):
        if exact:
            # lucky breakdown: the space holds every shifted solution
            di = np.linalg.solve(H[:p, :] - sigmas[i] * np.eye(p), beta[i] * c[:p])
            bi = 0.0
        else:
            M = np.hstack([H - sigmas[i] * Ib, s[:, None]])
            sol = np.linalg.solve(M, beta[i] * c)
            di, bi = sol[:p], sol[p]
        ds.append(di)
        beta_new[i] = bi
    return ds, s, beta_new


def fom_small_solves(H, c, sigmas, beta):
    """FOM-Sh small problems (Sec. 3, Examples 2-3): the Galerkin conditions
    (H_m - sigma_i I) y_i = beta_i c_{1:m} on the square part of the
    recurrence. Every residual is then a multiple of v_{m+1},
    r_i = -h_{m+1,m} (e_m^T y_i) v_{m+1}, so the residuals of all shifts are
    parallel without any extra condition. Same return shape as
    shifted_small_solves: (ys, s, beta_new) with s = c - (H_bar - sigma_1 I_bar) y_1."""
    p = H.shape[1]
    Hm = H[:p, :]
    Ip = np.eye(p, dtype=np.complex128)
    ys = [np.linalg.solve(Hm - sigmas[i] * Ip, beta[i] * c[:p]) for i in range(len(sigmas))]
    s = c - (H - sigmas[0] * ibar(p + 1, p)) @ ys[0]
    beta_new = np.ones(len(sigmas), dtype=np.complex128)
    for i in range(1, len(sigmas)):
        beta_new[i] = ys[i][p - 1] / ys[0][p - 1]
    return ys, s, beta_new


def ritz(H, sigma1):
    """Ritz values/vectors of the base-shifted square part H_m - sigma_1 I
    (the deflation of FOM-DR)."""
    m = H.shape[1]
    return np.linalg.eig(H[:m, :] - sigma1 * np.eye(m, dtype=np.complex128))


# ----------------------------------------------------------------------------
# GMRES-DR restart: harmonic Ritz deflation (eqs. (2.7)-(2.9))
# ----------------------------------------------------------------------------
def harmonic_ritz(H, sigma1):
    """Harmonic Ritz values/vectors of the base-shifted (m+1) x m H_bar."""
    m = H.shape[1]
    Hs = H - sigma1 * ibar(m + 1, m)
    Hm = Hs[:m, :]
    em = np.zeros(m, dtype=np.complex128)
    em[m - 1] = 1.0
    f = np.linalg.solve(Hm.conj().T, em)
    G = Hm + abs(Hs[m, m - 1]) ** 2 * np.outer(f, em)
    theta, g = np.linalg.eig(G)
    return theta, g


def select_smallest(theta, k, rtol=1e-10):
    """Indices of the k smallest |theta|, in that order; ties by smaller Re,
    then smaller Im. Moduli and real parts equal to a relative rtol count as
    ties: for real data the harmonic Ritz values come in conjugate pairs whose
    computed moduli differ only by rounding, and the pair is then ordered by
    the sign of Im (negative first) instead of by rounding noise."""
    def less(a, b):
        ma, mb = abs(a), abs(b)
        tol = rtol * max(ma, mb)
        if abs(ma - mb) > tol:
            return ma < mb
        if abs(a.real - b.real) > tol:
            return a.real < b.real
        return a.imag < b.imag
    rest = list(range(len(theta)))
    out = []
    for _ in range(min(k, len(rest))):
        best = rest[0]
        for j in rest[1:]:
            if less(theta[j], theta[best]):
                best = j
        out.append(best)
        rest.remove(best)
    return np.array(out, dtype=int)


def dr_restart(V, H, s, sigma1, k, fom=False):
    """Compress V_{m+1}, H_bar_m to V_{k+1}, H_bar_k around k harmonic Ritz
    vectors (Ritz vectors for FOM-DR) and the residual direction s. Returns
    (V_{k+1}, H_bar_k, c_new, selected theta)."""
    m = H.shape[1]
    P = np.zeros((m + 1, k + 1), dtype=np.complex128)
    theta_sel = np.zeros(0, dtype=np.complex128)
    if k > 0:
        theta, g = ritz(H, sigma1) if fom else harmonic_ritz(H, sigma1)
        sel = select_smallest(theta, k)
        theta_sel = theta[sel]
        Pk, _ = np.linalg.qr(g[:, sel])
        P[:m, :k] = Pk
    p = s.copy()
    for _ in range(2):
        p = p - P[:, :k] @ (P[:, :k].conj().T @ p)
    P[:, k] = p / norm(p)
    Hk = P.conj().T @ H @ P[:m, :k]
    Vk1 = V @ P
    v = Vk1[:, k]
    for _ in range(2):
        v = v - Vk1[:, :k] @ (Vk1[:, :k].conj().T @ v)
    Vk1[:, k] = v / norm(v)
    c_new = P.conj().T @ s
    return Vk1, Hk, c_new, theta_sel


# ----------------------------------------------------------------------------
# GMRES-DR-Sh (Sec. 3, algorithm GMRES-DR-Sh)
# ----------------------------------------------------------------------------
def gmres_dr_sh(matvec, b, sigmas, m, k, tol, max_cycles=500, fom=False):
    """Solve (A - sigma_i I) x_i = b for all shifts in one deflated space.
    fom: FOM-DR-Sh instead (Galerkin small problems, Ritz deflation; Sec. 3,
    Example 3); with k = 0 this is FOM(m)-Sh / GMRES(m)-Sh.

    Returns a dict: x (ns, n), beta, cycles, mvps, converged, history (per
    cycle: mvps, ||r_1||/||b||, max_i |beta_i| ||r_1||/||b||, selected
    theta), defl = (V_{k+1}, H_bar_k) or None.
    """
    if not (m > k >= 0):
        raise ValueError("need m > k >= 0")
    sigmas = np.asarray(sigmas, dtype=np.complex128)
    ns = len(sigmas)
    b = np.asarray(b, dtype=np.complex128)
    n = b.size
    bnorm = norm(b)
    x = np.zeros((ns, n), dtype=np.complex128)
    beta = np.ones(ns, dtype=np.complex128)
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    c = np.zeros(m + 1, dtype=np.complex128)
    V[:, 0] = b / bnorm
    c[0] = bnorm
    j0 = 0
    mvps = 0
    history = []
    converged = False
    defl = None
    cycles = 0
    for cycle in range(max_cycles):
        cycles += 1
        mdim = m
        for j in range(j0, m):
            mvps += 1
            if arnoldi_step(matvec, V, H, j):
                mdim = j + 1
                break
        small = fom_small_solves if fom else shifted_small_solves
        ds, s, beta_new = small(H[:mdim + 1, :mdim], c[:mdim + 1], sigmas, beta)
        for i in range(ns):
            x[i] += V[:, :mdim] @ ds[i]
        beta = beta_new
        rnorm = norm(s)
        res = np.abs(beta) * rnorm / bnorm
        converged = bool(np.max(res) <= tol) or mdim < m
        entry = dict(cycle=cycles, mvps=mvps, r1=rnorm / bnorm,
                     rmax=float(np.max(res)), res=res.copy(), theta=None)
        if mdim < m:
            history.append(entry)
            break
        Vk1, Hk, c_k, theta = dr_restart(V, H, s, sigmas[0], k, fom=fom)
        entry["theta"] = theta
        history.append(entry)
        if converged:
            defl = (Vk1.copy(), Hk.copy())
            break
        V[:] = 0
        H[:] = 0
        c[:] = 0
        V[:, :k + 1] = Vk1
        H[:k + 1, :k] = Hk
        c[:k + 1] = c_k
        j0 = k
    return dict(x=x, beta=beta, cycles=cycles, mvps=mvps, converged=converged,
                history=history, defl=defl)


# ----------------------------------------------------------------------------
# Minres projection over V_k with v_{k+1} tracking (Sec. 2.3, Sec. 4)
# ----------------------------------------------------------------------------
def minres_projection_sh(Vk1, Hk, sigmas, x, r1, beta, gam):
    """Project the base system over span(V_k) by minimum residual, and move
    the other shifts so that r_i = beta_i r_1 + gamma_i v_{k+1} (eqs.
    (4.1)-(4.2)). Updates x and gam in place; returns the new r_1."""
    k = Hk.shape[1]
    Vk = Vk1[:, :k]
    c = Vk1.conj().T @ r1
    Hk1 = Hk - sigmas[0] * ibar(k + 1, k)
    d1 = np.linalg.lstsq(Hk1, c, rcond=None)[0]
    x[0] += Vk @ d1
    r1 = r1 - Vk1 @ (Hk1 @ d1)
    Hkk = Hk[:k, :]
    Ik = np.eye(k, dtype=np.complex128)
    for i in range(1, len(sigmas)):
        t = beta[i] * ((Hkk - sigmas[0] * Ik) @ d1)
        di = np.linalg.solve(Hkk - sigmas[i] * Ik, t)
        x[i] += Vk @ di
        gam[i] += Hk[k, :] @ (beta[i] * d1 - di)
    return r1


def leading_projection_sh(Vk1, Hk, sigmas, x, r1, beta, kp):
    """Projection over the most accurate approximate eigenvectors only
    (Sec. 4, Theorem 1 and Example 4 / Table 4.1). The leading kp columns of
    V_k span the kp approximate eigenvectors of smallest harmonic Ritz value
    (the restart keeps them in that order), and A V_kp = V_{k+1} Hbar_k[:, :kp].
    Base shift: minimum residual over span(V_kp). Other shifts: the first kp
    rows of (H - sigma_i I) d_i = beta_i (H - sigma_1 I) d_1, i.e. step 4 of
    GMRES-Proj-Sh on the kp-column recurrence; beta_i is unchanged and the
    residuals stay parallel only for exact eigenvectors (Theorem 1). Updates x
    in place; returns the new r_1."""
    k = Hk.shape[1]
    Vkp = Vk1[:, :kp]
    c = Vk1.conj().T @ r1
    Hs = (Hk - sigmas[0] * ibar(k + 1, k))[:, :kp]
    d1 = np.linalg.lstsq(Hs, c, rcond=None)[0]
    x[0] += Vkp @ d1
    r1 = r1 - Vk1 @ (Hs @ d1)
    Hkk = Hk[:kp, :kp]
    Ik = np.eye(kp, dtype=np.complex128)
    for i in range(1, len(sigmas)):
        t = beta[i] * ((Hkk - sigmas[0] * Ik) @ d1)
        di = np.linalg.solve(Hkk - sigmas[i] * Ik, t)
        x[i] += Vkp @ di
    return r1


def gmres_sh_cycle(matvec, x, r1, beta, sigmas, m):
    """One cycle of GMRES(m)-Sh from the current base residual r_1, the
    other shifts holding residuals beta_i r_1 (Sec. 2.1). The new base
    residual is formed recursively as V_{m+1} s (no extra products).
    Returns (r_1, beta_new, matrix-vector products used)."""
    n = r1.size
    V = np.zeros((n, m + 1), dtype=np.complex128)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    c = np.zeros(m + 1, dtype=np.complex128)
    rn = norm(r1)
    V[:, 0] = r1 / rn
    c[0] = rn
    mdim = m
    for j in range(m):
        if arnoldi_step(matvec, V, H, j):
            mdim = j + 1
            break
    ds, s, beta_new = shifted_small_solves(H[:mdim + 1, :mdim], c[:mdim + 1],
                                           sigmas, beta)
    for i in range(len(sigmas)):
        x[i] += V[:, :mdim] @ ds[i]
    r1 = V[:, :mdim + 1] @ s
    return r1, beta_new, mdim


def gmres_proj_sh(matvec, b, sigmas, defl, m, tol, max_cycles=500, x0=None,
                  r0=None, kp=None):
    """GMRES(m)-Proj(k)-Sh for one right-hand side (Sec. 4, steps 2-6):
    alternate the projection over V_k with one GMRES(m)-Sh cycle until the
    base residual and every |beta_i| ||r_1|| are below tol ||b|| (the
    component along v_{k+1} is ignored here and removed by the correction).

    x0/r0 allow a start from a common-residual initial guess (Sec. 5).
    kp: project over the leading kp deflation vectors only, the accurate
    eigenvector variant of Table 4.1 (no v_{k+1} tracking).
    Returns dict with x, beta, gam, r1, mvps, cycles, converged, history.
    """
    Vk1, Hk = defl
    sigmas = np.asarray(sigmas, dtype=np.complex128)
    ns = len(sigmas)
    b = np.asarray(b, dtype=np.complex128)
    bnorm = norm(b)
    x = np.zeros((ns, b.size), dtype=np.complex128) if x0 is None else x0.copy()
    r1 = b.copy() if r0 is None else r0.copy()
    beta = np.ones(ns, dtype=np.complex128)
    gam = np.zeros(ns, dtype=np.complex128)
    mvps = 0
    history = []
    converged = False
    cycles = 0
    for _ in range(max_cycles):
        cycles += 1
        if kp is None:
            r1 = minres_projection_sh(Vk1, Hk, sigmas, x, r1, beta, gam)
        else:
            r1 = leading_projection_sh(Vk1, Hk, sigmas, x, r1, beta, kp)
        r1, beta, used = gmres_sh_cycle(matvec, x, r1, beta, sigmas, m)
        mvps += used
        rn = norm(r1)
        res = np.abs(beta) * rn / bnorm
        history.append(dict(cycle=cycles, mvps=mvps, r1=rn / bnorm,
                            rmax=float(np.max(res)), gam=gam.copy()))
        if np.max(res) <= tol:
            converged = True
            break
    return dict(x=x, beta=beta, gam=gam, r1=r1, mvps=mvps, cycles=cycles,
                converged=converged, history=history)


# ----------------------------------------------------------------------------
# Extra right-hand side v_{k+1} and the correction phase (eqs. (4.3)-(4.6))
# ----------------------------------------------------------------------------
def true_residual(matvec, b, x, sigma):
    return b - (matvec(x) - sigma * x)


def extra_rhs(matvec, sigmas, defl, m, tol_extra, max_cycles=500):
    """Solve (A - sigma_i I) s_i = v_{k+1} for i >= 2: GMRES-Proj-Sh, then
    s_i = s~_i / (1 - gamma_i), gamma_i = v_{k+1}^H (v_{k+1} - (A - sigma_i) s~_i)."""
    Vk1, _ = defl
    v = Vk1[:, -1]
    out = gmres_proj_sh(matvec, v, sigmas, defl, m, tol_extra, max_cycles)
    s = out["x"].copy()
    gam_hat = np.zeros(len(sigmas), dtype=np.complex128)
    for i in range(1, len(sigmas)):
        r = true_residual(matvec, v, s[i], sigmas[i])
        gam_hat[i] = np.vdot(v, r)
        s[i] = s[i] / (1.0 - gam_hat[i])
    out["s"] = s
    out["gam_hat"] = gam_hat
    return out


def correct(matvec, b, x, sigmas, vk1, s):
    """x_i <- x_i + (v_{k+1}^H r_i) s_i for i >= 2, r_i the true residual."""
    gam_hat = np.zeros(len(sigmas), dtype=np.complex128)
    for i in range(1, len(sigmas)):
        r = true_residual(matvec, b, x[i], sigmas[i])
        gam_hat[i] = np.vdot(vk1, r)
        x[i] = x[i] + gam_hat[i] * s[i]
    return gam_hat


# ----------------------------------------------------------------------------
# Related right-hand sides (Sec. 5)
# ----------------------------------------------------------------------------
def related_rhs_start(B, X, b):
    """Minres projection over earlier solutions: B^H B d = B^H b (shift
    independent), x~_i = X_i d, common residual b - B d.
    B is (n, j-1), X is (ns, n, j-1)."""
    d = np.linalg.solve(B.conj().T @ B, B.conj().T @ b)
    x0 = np.einsum("inj,j->in", X, d)
    return x0, b - B @ d


# ----------------------------------------------------------------------------
# Driver: first RHS by GMRES-DR-Sh, extra RHS, later RHS by GMRES-Proj-Sh
# ----------------------------------------------------------------------------
def solve_all(matvec, B, sigmas, m_dr, k, m_proj, tol, tol_extra,
              max_cycles=500, related=False, fom=False):
    """Order of use (Sec. 4): RHS 1 by GMRES-DR-Sh, then the extra RHS
    v_{k+1}, then RHS 2.. by GMRES-Proj-Sh followed by the correction.
    fom: RHS 1 by FOM-DR-Sh instead; its (V_{k+1}, H_bar_k) satisfies the
    same recurrence, so the later right-hand sides are unchanged.

    Returns dict with X (nrhs, ns, n), per-RHS run records, the deflation
    pair, the extra-RHS solutions s and the true residual norms
    resid[j, i] = ||b^j - (A - sigma_i) x_i^j|| / ||b^j||.
    """
    sigmas = np.asarray(sigmas, dtype=np.complex128)
    B = np.asarray(B, dtype=np.complex128)
    nrhs, n = B.shape
    ns = len(sigmas)
    X = np.zeros((nrhs, ns, n), dtype=np.complex128)
    runs = []
    first = gmres_dr_sh(matvec, B[0], sigmas, m_dr, k, tol, max_cycles, fom=fom)
    X[0] = first["x"]
    runs.append(first)
    defl = first["defl"]
    extra = None
    if nrhs > 1:
        if defl is None:
            raise RuntimeError("no deflation pair: first solve ended early")
        extra = extra_rhs(matvec, sigmas, defl, m_proj, tol_extra, max_cycles)
        vk1 = defl[0][:, -1]
        for j in range(1, nrhs):
            x0 = r0 = None
            if related:
                x0, r0 = related_rhs_start(B[:j].T, X[:j].transpose(1, 2, 0), B[j])
            out = gmres_proj_sh(matvec, B[j], sigmas, defl, m_proj, tol,
                                max_cycles, x0=x0, r0=r0)
            out["gam_hat"] = correct(matvec, B[j], out["x"], sigmas, vk1, extra["s"])
            X[j] = out["x"]
            runs.append(out)
    resid = np.zeros((nrhs, ns))
    for j in range(nrhs):
        bn = norm(B[j])
        for i in range(ns):
            resid[j, i] = norm(true_residual(matvec, B[j], X[j, i], sigmas[i])) / bn
    return dict(X=X, runs=runs, defl=defl, extra=extra, resid=resid)
