// Small dense FP64 problems of a restart cycle, on the device.
//
// One 64-lane wavefront per problem, matrices in LDS (column-major, odd
// leading dimension so that both row- and column-strided lane accesses are
// bank-conflict free). Per cycle (Sec. 2.1 and the GMRES-DR-Sh algorithm):
//   * base shift: min ||c - (H_bar - sigma_1 I_bar) d_1|| by Householder QR,
//     s = c - (H_bar - sigma_1 I_bar) d_1;
//   * shift i >= 2: QR of H_bar - sigma_i I_bar applied to c and s; the last
//     row fixes beta_i^new = beta_i (Q^H c)_{m+1} / (Q^H s)_{m+1}, the first
//     m rows give d_i by back substitution;
//   * GMRES-DR restart (block 0): harmonic Ritz values of the base-shifted
//     matrix as the eigenvalues of G = H_m + |h_{m+1,m}|^2 H_m^{-H} e_m e_m^H
//     (Hessenberg reduction, then complex shifted-QR Schur form
//     G = Z T Z^H); the k eigenvalues of smallest |theta| (ties by Re, then
//     Im) are moved to the top of T by adjacent Givens swaps, so the first k
//     Schur vectors are an orthonormal basis of their eigenvectors' span.
//     P_{k+1} = [Z_k; 0 | s orthogonalised against them], H_bar_new =
//     P_{k+1}^H H_bar P_k, c_new = P_{k+1}^H s.
// Projection step of GMRES-Proj-Sh (Sec. 4): min ||c - (H_bar_k - sigma_1
// I_bar) d_1||, then (H_k - sigma_i I) d_i = beta_i (H_k - sigma_1 I) d_1 and
// gamma_i += h_{k+1,:} (beta_i d_1 - d_i) (eq. (4.2)).
#include "small.h"

namespace gdr {

constexpr int LD = 65;
#define AT(M, r, c) (M)[(c) * LD + (r)]

__device__ __forceinline__ double wred(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ double2 csqrt_(double2 z) {
    double r = cabs(z);
    double a = sqrt(fmax(0.5 * (r + z.x), 0.0));
    double b = sqrt(fmax(0.5 * (r - z.x), 0.0));
    return mk(a, z.y < 0 ? -b : b);
}

// lexicographic key (|theta|, Re, Im)
// Selection order of harmonic Ritz values: smaller |theta|, then smaller
// Re theta, then smaller Im theta, where moduli and real parts equal to a
// relative 1e-10 count as ties (for real data the values come in conjugate
// pairs whose computed moduli differ only by rounding; the tie then goes to
// the member with negative imaginary part).
__device__ __forceinline__ bool key_less(double2 a, double2 b) {
    const double aa = cabs(a), ab = cabs(b);
    const double tol = 1e-10 * fmax(aa, ab);
    if (fabs(aa - ab) > tol) return aa < ab;
    if (fabs(a.x - b.x) > tol) return a.x < b.x;
    return a.y < b.y;
}

// Householder QR of the first `cols` columns of the rows x ctot LDS matrix A;
// the remaining columns receive Q^H. R is left in the upper triangle.
// Column j may be nonzero down to row max(j + 1, band) only (band = rows:
// dense): an upper Hessenberg matrix whose leading block is dense down to
// row band, as the cycle's H_bar after a restart to band deflation vectors.
// The reflector of column j then has nonzeros in rows j..max(j + 1, band)
// only, and the loops stop there (the rows below hold exact zeros, so the
// result is that of the dense loops).
__device__ void hh_qr(double2* A, int rows, int cols, int ctot, double2* hv, int band) {
    const int lane = threadIdx.x;
    for (int j = 0; j < cols && j < rows; ++j) {
        const int end = min(rows, max(j + 2, band + 1));   // rows j..end-1
        double ss = 0;
        for (int r = j + lane; r < end; r += 64) ss += cabs2(AT(A, r, j));
        ss = wred(ss);
        const double alpha = sqrt(ss);
        const double2 x0 = AT(A, j, j);
        const double ax0 = cabs(x0);
        __syncthreads();
        if (!(alpha > 0.0)) continue;
        const double2 ph = ax0 > 0 ? cscale(x0, 1.0 / ax0) : mk(1, 0);
        for (int r = j + lane; r < end; r += 64)
            hv[r] = (r == j) ? cadd(x0, cscale(ph, alpha)) : AT(A, r, j);
        const double tau = 1.0 / (alpha * (alpha + ax0));   // 2 / ||v||^2
        __syncthreads();
        for (int c = j + 1 + lane; c < ctot; c += 64) {
            double2 d = mk(0, 0);
            for (int r = j; r < end; ++r) d = cadd(d, cjmul(hv[r], AT(A, r, c)));
            d = cscale(d, tau);
            for (int r = j; r < end; ++r) AT(A, r, c) = csub(AT(A, r, c), cmul(hv[r], d));
        }
        for (int r = j + lane; r < end; r += 64) AT(A, r, j) = (r == j) ? cscale(ph, -alpha) : mk(0, 0);
        __syncthreads();
    }
}

// Solve R y = y in place (R upper triangular nn x nn in A). Returns false if
// a pivot is zero or tiny relative to the largest.
__device__ bool back_sub(const double2* A, int nn, double2* y) {
    const int lane = threadIdx.x;
    double rmax = 0;
    for (int j = 0; j < nn; ++j) rmax = fmax(rmax, cabs(AT(A, j, j)));
    bool ok = true;
    for (int j = nn - 1; j >= 0; --j) {
        __syncthreads();
        const double2 piv = AT(A, j, j);
        if (!(cabs(piv) > 1e-14 * rmax)) ok = false;
        const double2 dj = cdiv(y[j], piv);
        __syncthreads();
        if (lane == 0) y[j] = dj;
        for (int r = lane; r < j; r += 64) y[r] = csub(y[r], cmul(AT(A, r, j), dj));
    }
    __syncthreads();
    return ok;
}

__device__ __forceinline__ void givens(double2 x, double2 y, double& c, double2& s) {
    const double ax = cabs(x), ay = cabs(y);
    if (ay == 0.0) {
        c = 1.0;
        s = mk(0, 0);
    } else if (ax == 0.0) {
        c = 0.0;
        s = cscale(cconj(y), 1.0 / ay);
    } else {
        const double rho = hypot(ax, ay);
        c = ax / rho;
        s = cscale(cmul(cscale(x, 1.0 / ax), cconj(y)), 1.0 / rho);
    }
}

// rows p, p+1, columns [c0, c1): [rp; rq] <- [[c, s], [-conj(s), c]] [rp; rq]
__device__ __forceinline__ void rot_rows(double2* M, int p, int c0, int c1, double c, double2 s) {
    for (int col = c0 + (int)threadIdx.x; col < c1; col += 64) {
        const double2 a = AT(M, p, col), b = AT(M, p + 1, col);
        AT(M, p, col) = cadd(cscale(a, c), cmul(s, b));
        AT(M, p + 1, col) = csub(cscale(b, c), cjmul(s, a));
    }
}
// columns p, p+1, rows [r0, r1): M <- M G^H
__device__ __forceinline__ void rot_cols(double2* M, int p, int r0, int r1, double c, double2 s) {
    for (int r = r0 + (int)threadIdx.x; r < r1; r += 64) {
        const double2 a = AT(M, r, p), b = AT(M, r, p + 1);
        AT(M, r, p) = cadd(cscale(a, c), cjmul(s, b));
        AT(M, r, p + 1) = csub(cscale(b, c), cmul(s, a));
    }
}

// Reduce T (nn x nn) to upper Hessenberg form by Householder similarity,
// accumulating Z <- Z H (Z enters as the identity).
__device__ void hessenberg(double2* T, double2* Z, int nn, double2* hv) {
    const int lane = threadIdx.x;
    for (int j = 0; j + 2 < nn; ++j) {
        double ss = 0;
        for (int r = j + 1 + lane; r < nn; r += 64) ss += cabs2(AT(T, r, j));
        ss = wred(ss);
        const double2 x0 = AT(T, j + 1, j);
        const double ax0 = cabs(x0);
        const double tail = ss - ax0 * ax0;
        const double alpha = sqrt(ss);
        __syncthreads();
        if (!(tail > 0.0)) continue;   // already Hessenberg in this column
        const double2 ph = ax0 > 0 ? cscale(x0, 1.0 / ax0) : mk(1, 0);
        for (int r = j + 1 + lane; r < nn; r += 64)
            hv[r] = (r == j + 1) ? cadd(x0, cscale(ph, alpha)) : AT(T, r, j);
        const double tau = 1.0 / (alpha * (alpha + ax0));
        __syncthreads();
        // left: T[j+1:, j:] -= tau v (v^H T)
        for (int c = j + lane; c < nn; c += 64) {
            double2 d = mk(0, 0);
            for (int r = j + 1; r < nn; ++r) d = cadd(d, cjmul(hv[r], AT(T, r, c)));
            d = cscale(d, tau);
            for (int r = j + 1; r < nn; ++r) AT(T, r, c) = csub(AT(T, r, c), cmul(hv[r], d));
        }
        __syncthreads();
        // right: T[:, j+1:] -= tau (T v) v^H ; Z likewise
        for (int r = lane; r < nn; r += 64) {
            double2 d = mk(0, 0), e = mk(0, 0);
            for (int c = j + 1; c < nn; ++c) {
                d = cadd(d, cmul(AT(T, r, c), hv[c]));
                e = cadd(e, cmul(AT(Z, r, c), hv[c]));
            }
            d = cscale(d, tau);
            e = cscale(e, tau);
            for (int c = j + 1; c < nn; ++c) {
                AT(T, r, c) = csub(AT(T, r, c), cmul(d, cconj(hv[c])));
                AT(Z, r, c) = csub(AT(Z, r, c), cmul(e, cconj(hv[c])));
            }
        }
        __syncthreads();
        for (int r = j + 2 + lane; r < nn; r += 64) AT(T, r, j) = mk(0, 0);
        __syncthreads();
    }
}

// 1/sqrt(a) for normal a > 0: the hardware estimate refined by two Newton
// steps y <- y (3 - a y^2) / 2 (quadratic convergence to full precision).
__device__ __forceinline__ double rsqrt_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
    y = y * (1.5 - 0.5 * a * y * y);
    y = y * (1.5 - 0.5 * a * y * y);
    return y;
}

// Givens parameters (the small matrices are well scaled):
// [[c, s], [-conj(s), c]] [x; y] = [r; 0], c real >= 0.
__device__ __forceinline__ void givens_fast(double2 x, double2 y, double& c, double2& s) {
    const double ax2 = cabs2(x), ay2 = cabs2(y);
    if (ay2 == 0.0) {
        c = 1.0;
        s = mk(0, 0);
    } else if (ax2 == 0.0) {
        c = 0.0;
        s = cscale(cconj(y), rsqrt_nr(ay2));
    } else {
        const double iax = rsqrt_nr(ax2);
        const double ir = rsqrt_nr(ax2 + ay2);
        c = ax2 * iax * ir;
        s = cscale(cmul(x, cconj(y)), ir * iax);
    }
}

// The small kernels run one wavefront per workgroup: a wave-local fence is
// enough to order LDS writes before other lanes' reads.
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Apply the rotations kk = k0..k1-1 (parameters rc/rs[kk]) to columns
// kk, kk+1 of row r of M, in order, carrying the running entry. Runs of 8
// rotations load their row entries and parameters first: rotation kk reads
// column kk+1 and writes column kk, so no entry a run reads was written in
// it, and the loads are not each waited for in turn.
__device__ __forceinline__ void rot_row_seq(double2* M, int r, int k0, int k1, const double* rc,
                                            const double2* rs) {
    if (k0 >= k1) return;
    double2 a = AT(M, r, k0);
    int kk = k0;
    for (; kk + 8 <= k1; kk += 8) {
        double2 b[8], sv[8];
        double c[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            b[t] = AT(M, r, kk + 1 + t);
            c[t] = rc[kk + t];
            sv[t] = rs[kk + t];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            AT(M, r, kk + t) = cadd(cscale(a, c[t]), cjmul(sv[t], b[t]));
            a = csub(cscale(b[t], c[t]), cmul(sv[t], a));
        }
    }
    for (; kk < k1; ++kk) {
        const double2 b = AT(M, r, kk + 1);
        const double c = rc[kk];
        const double2 sv = rs[kk];
        AT(M, r, kk) = cadd(cscale(a, c), cjmul(sv, b));
        a = csub(cscale(b, c), cmul(sv, a));
    }
    AT(M, r, k1) = a;
}

// value of v in lane l (l uniform), through scalar registers
__device__ __forceinline__ double rlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 rlane2(double2 v, int l) { return mk(rlane(v.x, l), rlane(v.y, l)); }

// Complex Schur form of the upper Hessenberg T (nn <= 64) by single-shift QR
// with Wilkinson shifts; Z accumulates. A bulge-chase sweep runs one lane per
// column: lane c carries the current value of its column in the row being
// rotated, applies each left rotation to it (writing the finished upper row)
// and reads the next row's value, so the sweep needs no LDS round trip or
// barrier between rotations. A right rotation kk is applied at once only to
// rows kk+1 and kk+2 (the values the next rotations are computed from, taken
// from lanes kk and kk+1); its updates of the rows above and of Z follow
// after the sweep, row by row in rotation order (left and right rotations
// commute, and every entry receives its rotations of each side in order, so
// the result is the same similarity). Returns 0 on success.
__device__ int schur(double2* T, double2* Z, int nn, double* rc, double2* rs, long long* nrot) {
    const int lane = threadIdx.x;
    const double eps = 2.220446049250313e-16;
    double fro = 0;
    for (int c = 0; c < nn; ++c)
        for (int r = lane; r < nn; r += 64) fro += cabs2(AT(T, r, c));
    fro = sqrt(wred(fro));
    wsync();
    int hi = nn - 1, iter = 0, total = 0;
    while (hi > 0) {
        if (total > 60 * nn) return 1;
        // deflation test on squared magnitudes: |t_{l,l-1}|^2 <= eps^2 (|t_{l-1,l-1}|^2 + |t_{l,l}|^2);
        // lane l tests subdiagonal entry l, and l is the largest l <= hi that
        // passes (0 if none)
        bool negl = false;
        if (lane >= 1 && lane <= hi) {
            double tst = cabs2(AT(T, lane - 1, lane - 1)) + cabs2(AT(T, lane, lane));
            if (tst == 0.0) tst = fro * fro;
            negl = cabs2(AT(T, lane, lane - 1)) <= eps * eps * tst;
        }
        const unsigned long long bal = __ballot(negl);
        const int l = bal ? 63 - __clzll((long long)bal) : 0;
        wsync();
        if (l > 0 && lane == 0) AT(T, l, l - 1) = mk(0, 0);
        wsync();
        if (l == hi) {
            --hi;
            iter = 0;
            continue;
        }
        const int lo = l;
        double2 mu;
        if (iter > 0 && iter % 10 == 0) {
            mu = cadd(AT(T, hi, hi), mk(0.75 * cabs(AT(T, hi, hi - 1)), 0));
        } else {
            const double2 a = AT(T, hi - 1, hi - 1), b = AT(T, hi - 1, hi);
            const double2 cc = AT(T, hi, hi - 1), d = AT(T, hi, hi);
            const double2 half = cscale(csub(a, d), 0.5);
            const double2 sq = csqrt_(cadd(cmul(half, half), cmul(b, cc)));
            const double2 mid = cscale(cadd(a, d), 0.5);
            const double2 e1 = cadd(mid, sq), e2 = csub(mid, sq);
            mu = cabs(csub(e1, d)) <= cabs(csub(e2, d)) ? e1 : e2;
        }
        const int col = lane;
        const bool incol = col < nn && col >= lo;
        double2 carry = incol ? AT(T, lo, col) : mk(0, 0);   // row kk of column col
        double2 nxt = incol ? AT(T, lo + 1, col) : mk(0, 0);   // row kk+1 of column col
        double2 x = csub(AT(T, lo, lo), mu), y = AT(T, lo + 1, lo);
        // row kk+2 is untouched until rotation kk+2 (and the right rotations
        // wait for the end of the sweep): its subdiagonal entry and the values
        // of the columns right of it are loaded one rotation ahead
        double2 b2n = lo + 2 <= hi ? AT(T, lo + 2, lo + 1) : mk(0, 0);
        double2 pren = (lo + 2 <= hi && col < nn && col >= lo + 2) ? AT(T, lo + 2, col) : mk(0, 0);
        for (int kk = __builtin_amdgcn_readfirstlane(lo); kk < hi; ++kk) {
            const double2 b2 = b2n, pre = pren;
            const bool three = kk + 3 <= hi;
            b2n = three ? AT(T, kk + 3, kk + 2) : mk(0, 0);
            pren = (three && col < nn && col >= kk + 3) ? AT(T, kk + 3, col) : mk(0, 0);
            double c;
            double2 sv;
            givens_fast(x, y, c, sv);
            if (lane == 0) {
                rc[kk] = c;
                rs[kk] = sv;
            }
            // left rotation of rows kk, kk+1 (columns from kk-1; the
            // annihilated bulge entry becomes an exact zero)
            if (incol && col >= kk - 1) {
                const double2 a = carry, b = nxt;
                AT(T, kk, col) = cadd(cscale(a, c), cmul(sv, b));
                carry = (kk > lo && col == kk - 1) ? mk(0, 0) : csub(cscale(b, c), cjmul(sv, a));
            }
            // right rotation of columns kk, kk+1 in rows kk+1 (lanes kk, kk+1)
            // and kk+2 (zero and the subdiagonal entry: the new bulge)
            const double2 u = rlane2(carry, kk), v = rlane2(carry, kk + 1);
            const double2 u2 = cadd(cscale(u, c), cjmul(sv, v));
            const double2 v2 = csub(cscale(v, c), cmul(sv, u));
            const double2 bulge = cjmul(sv, b2), w2 = cscale(b2, c);
            if (col == kk) carry = u2;
            if (col == kk + 1) carry = v2;
            nxt = col == kk ? bulge : (col == kk + 1 ? w2 : pre);
            x = u2;
            y = bulge;
        }
        if (incol) AT(T, min(col + 2, hi), col) = carry;
        wsync();
        // deferred right rotations: row r < lo takes every rotation of the
        // sweep, row r in [lo, hi] the rotations kk >= r
        if (nrot && lane == 0) *nrot += hi - lo;
        for (int r = lane; r <= hi; r += 64) rot_row_seq(T, r, r < lo ? lo : r, hi, rc, rs);
        for (int r = lane; r < nn; r += 64) rot_row_seq(Z, r, lo, hi, rc, rs);
        wsync();
        ++iter;
        ++total;
    }
    return 0;
}

// swap the adjacent diagonal entries p, p+1 of the triangular T; the
// rotation is recorded in (rc, rs)[slot] for a later batched update of Z
__device__ void schur_swap(double2* T, int nn, int p, double* rc, double2* rs, int slot) {
    const double2 t11 = AT(T, p, p), t22 = AT(T, p + 1, p + 1), t12 = AT(T, p, p + 1);
    double c;
    double2 s;
    givens_fast(t12, csub(t22, t11), c, s);
    if (threadIdx.x == 0) {
        rc[slot] = c;
        rs[slot] = s;
    }
    wsync();
    rot_rows(T, p, p, nn, c, s);
    wsync();
    rot_cols(T, p, 0, p + 2, c, s);
    wsync();
    if (threadIdx.x == 0) {
        AT(T, p, p) = t22;
        AT(T, p + 1, p + 1) = t11;
        AT(T, p + 1, p) = mk(0, 0);
    }
    wsync();
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_cycle_small(CycleArgs a) {
    const int lane = threadIdx.x;
    const int role = blockIdx.x;   // 0: base (+ restart), i >= 1: shift i
    const int b = blockIdx.y;
    if (a.act && !a.act[b]) return;
    const int m = a.m;
    const int ns = a.ns;
    const double2* H = a.H + b * a.h_ms;
    const double2* cg = a.c + b * a.c_ms;
    const double2* sig = a.sigma + b * a.sig_ms;
    const double2* beta = a.beta + b * a.beta_ms;
    double2* coef = a.coef + b * a.coef_ms;
    CycleOut* out = a.out + b;
    double2* const Pm = a.P ? a.P + b * a.p_ms : nullptr;
    double2* const Hm = a.Hnew ? a.Hnew + b * a.hnew_ms : nullptr;
    double2* const Cm = a.cnew ? a.cnew + b * a.cnew_ms : nullptr;
    const int ldh = m + 1;
    const int brk = a.brk[b];
    const int p = brk >= 0 ? brk + 1 : m;   // columns of this cycle

    __shared__ double2 A[(MAXM + 2) * LD];
    __shared__ double2 Zs[MAXM * LD];
    __shared__ double2 hv[LD + 1], sv[LD + 1], dv[LD + 1], fv[LD + 1];
    __shared__ double rotc[MAXM];
    __shared__ double2 rots[MAXM];

    long long t_start = wall_clock64();
    const double2 s1 = sig[0];
    const bool restart_only = a.restart == 2;
    const bool fom = a.galerkin != 0;
    bool base_ok = true;
    double2 y1_last = mk(0, 0);
    if (!restart_only) {
        // ---- base system: [Hs | c], Hs = H - sigma_1 I_bar. GMRES: least
        // squares over all p+1 rows; FOM: the square Galerkin system (first p rows)
        const int rows = fom ? p : p + 1;
        for (int c = 0; c <= p; ++c)
            for (int r = lane; r < rows; r += 64) {
                double2 v = c < p ? H[c * ldh + r] : cg[r];
                if (c < p && r == c) v = csub(v, s1);
                AT(A, r, c) = v;
            }
        __syncthreads();
        hh_qr(A, rows, p, p + 1, hv, a.k);
        for (int r = lane; r < p; r += 64) dv[r] = AT(A, r, p);
        __syncthreads();
        base_ok = back_sub(A, p, dv);
        y1_last = dv[p - 1];
        // s = c - Hs d_1 (from the original entries)
        for (int r = lane; r <= p; r += 64) {
            double2 acc = cg[r];
            for (int c = 0; c < p; ++c) {
                double2 h = H[c * ldh + r];
                if (r == c) h = csub(h, s1);
                acc = csub(acc, cmul(h, dv[c]));
            }
            sv[r] = acc;
        }
    } else {
        // restart half of a split cycle: s was written by the least-squares half
        for (int r = lane; r <= p; r += 64) sv[r] = coef[ns * (m + 1) + r];
    }
    __syncthreads();
    double sn = 0, cn = 0;
    for (int r = lane; r <= p; r += 64) {
        sn += cabs2(sv[r]);
        cn += cabs2(cg[r]);
    }
    sn = sqrt(wred(sn));
    cn = sqrt(wred(cn));
    const bool exact = !(sn > 1e-14 * cn);
    __syncthreads();

    if (role == 0) {
        if (!restart_only) {
            for (int r = lane; r <= m; r += 64) {
                coef[r] = r < p ? dv[r] : mk(0, 0);
                coef[ns * (m + 1) + r] = r <= p ? sv[r] : mk(0, 0);
            }
            if (lane == 0) {
                out->snorm = sn;
                out->beta[0] = mk(1, 0);
                if (fom && !base_ok && !exact) atomicOr(&out->flags, 1);
            }
        }
        if (a.restart == 0 || exact || p < m) return;
        // ---------------- DR restart (harmonic Ritz pairs for GMRES, Ritz pairs
        // for FOM, of the base-shifted matrix)
        const int k = a.k;
        if (lane == 0) {
            out->tclk[0] = t_start;
            out->tclk[1] = wall_clock64();
        }
        __syncthreads();
        if (k > 0) {
        double h2 = 0;
        if (!fom) {
        // f = Hm^{-H} e_m :  A = [Hm^H | e_m]
        for (int c = 0; c <= m; ++c)
            for (int r = lane; r < m; r += 64) {
                double2 v;
                if (c < m) {
                    v = H[r * ldh + c];                       // Hm[c][r]
                    if (r == c) v = csub(v, s1);
                    v = cconj(v);
                } else {
                    v = mk(r == m - 1 ? 1.0 : 0.0, 0);
                }
                AT(A, r, c) = v;
            }
        __syncthreads();
        hh_qr(A, m, m, m + 1, hv, m);
        for (int r = lane; r < m; r += 64) fv[r] = AT(A, r, m);
        __syncthreads();
        back_sub(A, m, fv);
        h2 = cabs2(H[(m - 1) * ldh + m]);
        }  // !fom
        if (lane == 0) out->tclk[2] = wall_clock64();
        // G = Hm + h2 f e_m^H (GMRES) or Hm (FOM) into A (m x m); Z = I
        for (int c = 0; c < m; ++c)
            for (int r = lane; r < m; r += 64) {
                double2 v = H[c * ldh + r];
                if (r == c) v = csub(v, s1);
                if (!fom && c == m - 1) v = cadd(v, cscale(fv[r], h2));
                AT(A, r, c) = v;
                AT(Zs, r, c) = mk(r == c ? 1.0 : 0.0, 0);
            }
        __syncthreads();
        hessenberg(A, Zs, m, hv);
        if (lane == 0) out->tclk[3] = wall_clock64();
        long long nrot = 0;
        int fail = schur(A, Zs, m, rotc, rots, &nrot);
        if (lane == 0) out->tclk[7] = nrot;
        if (lane == 0) out->tclk[4] = wall_clock64();
        if (fail) {
            if (lane == 0) atomicOr(&out->flags, 2);
            return;
        }
        // selection: k smallest |theta| moved to the top, in order
        for (int pos = 0; pos < k; ++pos) {
            int best = pos;
            for (int j = pos + 1; j < m; ++j)
                if (key_less(AT(A, j, j), AT(A, best, best))) best = j;
            __syncthreads();
            // swaps q = best-1 .. pos; Z takes them in the same order afterwards
            for (int q = best - 1; q >= pos; --q) schur_swap(A, m, q, rotc, rots, q);
            for (int r = lane; r < m; r += 64) {
                for (int q = best - 1; q >= pos; --q) {
                    const double2 a = AT(Zs, r, q), b = AT(Zs, r, q + 1);
                    const double c = rotc[q];
                    const double2 sq = rots[q];
                    AT(Zs, r, q) = cadd(cscale(a, c), cjmul(sq, b));
                    AT(Zs, r, q + 1) = csub(cscale(b, c), cmul(sq, a));
                }
            }
            if (lane == 0) out->theta[pos] = AT(A, pos, pos);
            __syncthreads();
        }
        }  // k > 0
        if (lane == 0) out->tclk[5] = wall_clock64();
        // p_{k+1}: s orthogonalised twice against [Z_k; 0], normalised
        for (int rep = 0; rep < 2; ++rep) {
            for (int j = lane; j < k; j += 64) {
                double2 d = mk(0, 0);
                for (int r = 0; r < m; ++r) d = cadd(d, cjmul(AT(Zs, r, j), sv[r]));
                hv[j] = d;
            }
            __syncthreads();
            for (int r = lane; r < m; r += 64) {
                double2 acc = sv[r];
                for (int j = 0; j < k; ++j) acc = csub(acc, cmul(AT(Zs, r, j), hv[j]));
                sv[r] = acc;
            }
            __syncthreads();
        }
        double pn = 0;
        for (int r = lane; r <= m; r += 64) pn += cabs2(sv[r]);
        pn = sqrt(wred(pn));
        __syncthreads();
        for (int r = lane; r <= m; r += 64) dv[r] = cscale(sv[r], 1.0 / pn);   // p_{k+1}
        __syncthreads();
        // P to global
        for (int j = 0; j <= k; ++j)
            for (int r = lane; r <= m; r += 64)
                Pm[j * (m + 1) + r] = j < k ? (r < m ? AT(Zs, r, j) : mk(0, 0)) : dv[r];
        // Y = H P_k into A ((m+1) x k), H unshifted
        for (int r = lane; r <= m; r += 64)
            for (int j = 0; j < k; ++j) {
                double2 acc = mk(0, 0);
                for (int l = 0; l < m; ++l) acc = cadd(acc, cmul(H[l * ldh + r], AT(Zs, l, j)));
                AT(A, r, j) = acc;
            }
        __syncthreads();
        // Hnew = P^H Y ((k+1) x k), zero elsewhere; c_new = P^H s_orig
        for (int t = lane; t < (m + 1) * m; t += 64) Hm[t] = mk(0, 0);
        __syncthreads();
        for (int t = lane; t < (k + 1) * k; t += 64) {
            const int i = t % (k + 1), j = t / (k + 1);
            double2 acc = mk(0, 0);
            if (i < k) {
                for (int r = 0; r < m; ++r) acc = cadd(acc, cjmul(AT(Zs, r, i), AT(A, r, j)));
            } else {
                for (int r = 0; r <= m; ++r) acc = cadd(acc, cjmul(dv[r], AT(A, r, j)));
            }
            Hm[j * (m + 1) + i] = acc;
        }
        // original s: recompute from coef column (written above)
        for (int i = lane; i <= m; i += 64) {
            double2 acc = mk(0, 0);
            if (i < k) {
                for (int r = 0; r < m; ++r) acc = cadd(acc, cjmul(AT(Zs, r, i), coef[ns * (m + 1) + r]));
            } else if (i == k) {
                for (int r = 0; r <= m; ++r) acc = cadd(acc, cjmul(dv[r], coef[ns * (m + 1) + r]));
            }
            Cm[i] = acc;
        }
        if (lane == 0) out->tclk[6] = wall_clock64();
        return;
    }

    const int i = role;
    if (i >= ns) return;
    const double2 si = sig[i];
    const double2 bi = beta[i];
    if (fom) {
        // ---------------- shift `role`, FOM: (H_p - sigma_i I) y_i = beta_i c_{1:p};
        // r_i = -h_{p+1,p} (y_i)_p v_{p+1}, hence beta_i^new = (y_i)_p / (y_1)_p
        for (int c = 0; c <= p; ++c)
            for (int r = lane; r < p; r += 64) {
                double2 v = c < p ? H[c * ldh + r] : cmul(bi, cg[r]);
                if (c < p && r == c) v = csub(v, si);
                AT(A, r, c) = v;
            }
        __syncthreads();
        hh_qr(A, p, p, p + 1, hv, a.k);
        for (int r = lane; r < p; r += 64) dv[r] = AT(A, r, p);
        __syncthreads();
        bool bad = !back_sub(A, p, dv);
        double2 bnew = mk(0, 0);
        if (!exact) {
            if (!(cabs(y1_last) > 0)) bad = true;
            else bnew = cdiv(dv[p - 1], y1_last);
        }
        for (int r = lane; r <= m; r += 64) coef[i * (m + 1) + r] = r < p ? dv[r] : mk(0, 0);
        if (lane == 0) {
            out->beta[i] = bnew;
            if (bad) atomicOr(&out->flags, 1);
        }
        return;
    }
    // ---------------- shift `role`, GMRES: [H - sigma_i I_bar | c | s]
    for (int c = 0; c < p + 2; ++c)
        for (int r = lane; r <= p; r += 64) {
            double2 v;
            if (c < p) {
                v = H[c * ldh + r];
                if (r == c) v = csub(v, si);
            } else if (c == p) {
                v = cg[r];
            } else {
                v = sv[r];
            }
            AT(A, r, c) = v;
        }
    __syncthreads();
    hh_qr(A, p + 1, p, p + 2, hv, a.k);
    double2 bnew;
    bool bad = false;
    if (exact) {
        bnew = mk(0, 0);
    } else {
        const double2 qc = AT(A, p, p), qs = AT(A, p, p + 1);
        if (!(cabs(qs) > 1e-14 * sn)) bad = true;
        bnew = cmul(bi, cdiv(qc, qs));
    }
    for (int r = lane; r < p; r += 64)
        dv[r] = csub(cmul(bi, AT(A, r, p)), cmul(bnew, AT(A, r, p + 1)));
    __syncthreads();
    if (!back_sub(A, p, dv)) bad = true;
    for (int r = lane; r <= m; r += 64) coef[i * (m + 1) + r] = r < p ? dv[r] : mk(0, 0);
    if (lane == 0) {
        out->beta[i] = bnew;
        if (bad) atomicOr(&out->flags, 1);
    }
}

__global__ __launch_bounds__(64) void k_sstep_small(SstepArgs a) {
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    if (a.act && !a.act[b]) return;
    const int j = a.j, sb = a.sb, nc = j + 1 + sb;
    const double2* G = a.G + b * a.g_ms;
    double2* Ps = a.Psave + b * a.p_ms;
    double* zn = a.znorm + b * BLK_MAX;
    double2* coef = a.coef + b * a.coef_ms;
    double2* beta = coef + BLK_MAX * (MAXM + 1);
    __shared__ double2 Pc[(MAXM + 1) * BLK_MAX];  // projection of this sweep
    __shared__ double2 Ch[(MAXM + 1) * BLK_MAX];  // total projection C-hat
    __shared__ double2 G2[BLK_MAX * BLK_MAX];
    __shared__ double2 R[BLK_MAX * BLK_MAX];      // R[l*BLK_MAX + c], upper
    __shared__ double2 Ri[BLK_MAX * BLK_MAX];     // inverse of the leading nq x nq block
    __shared__ int sh_fi, sh_two;
    for (int t = lane; t < (j + 1) * BLK_MAX; t += 64) {
        const int c = t / BLK_MAX, q = t % BLK_MAX;
        const double2 p = q < sb ? G[q * nc + c] : mk(0, 0);
        Pc[t] = p;
        if (a.mode == 1) {
            Ps[t] = p;
            Ch[t] = p;
        } else {
            Ch[t] = q < sb ? cadd(Ps[t], p) : mk(0, 0);
        }
    }
    if (a.mode == 1 && lane < sb) zn[lane] = G[lane * nc + j + 1 + lane].x;
    __syncthreads();
    // Gram of the block with the V components of this sweep removed:
    // G2 = X^H X - Pc^H Pc (X = Z after the first sweep, Z' after the second)
    for (int e = 0; e < sb * sb; ++e) {
        const int r = e / sb, q = e % sb;
        double sx = 0, sy = 0;
        for (int c = lane; c <= j; c += 64) {
            const double2 v = cjmul(Pc[c * BLK_MAX + r], Pc[c * BLK_MAX + q]);
            sx += v.x;
            sy += v.y;
        }
        sx = wred(sx);
        sy = wred(sy);
        if (lane == 0) G2[r * BLK_MAX + q] = csub(G[q * nc + j + 1 + r], mk(sx, sy));
    }
    __syncthreads();
    if (lane == 0) {
        // one sweep suffices unless the projection cancelled much of a block
        // vector (its stored FP32 rounding then leaves V components behind)
        int two = 0;
        if (a.mode == 1) {
            for (int i = 0; i < sb; ++i) {
                const double g = G2[i * BLK_MAX + i].x;
                if (!(g > 0) || !(g * a.reorth > zn[i])) two = 1;
            }
            if (a.reorth <= 0) two = 1;
        }
        sh_two = two;
        if (a.reo) a.reo[b] = two;
    }
    __syncthreads();
    if (sh_two) {
        // intermediate update Z' = Z - V_{0..j} P1; the second sweep finishes
        for (int t = lane; t < (j + 1) * sb; t += 64) {
            const int c = t / sb, q = t % sb;
            coef[q * (MAXM + 1) + c] = Pc[c * BLK_MAX + q];
        }
        if (lane < BLK_MAX * BLK_MAX) beta[lane] = mk((lane / BLK_MAX) == (lane % BLK_MAX) ? 1.0 : 0.0, 0);
        return;
    }
    if (lane == 0) {
        int fi = -1;
        for (int t = 0; t < BLK_MAX * BLK_MAX; ++t) {
            R[t] = mk(0, 0);
            Ri[t] = mk(0, 0);
        }
        for (int i = 0; i < sb && fi < 0; ++i) {
            // row i of R: R[i][c] = (G2[i][c] - sum_{l<i} conj(R[l][i]) R[l][c]) / R[i][i]
            double piv = G2[i * BLK_MAX + i].x;
            for (int l = 0; l < i; ++l) piv -= cabs2(R[l * BLK_MAX + i]);
            if (!(piv > 1e-10 * zn[i])) {
                fi = i;
                break;
            }
            const double rii = sqrt(piv);
            R[i * BLK_MAX + i] = mk(rii, 0);
            for (int c = i + 1; c < sb; ++c) {
                double2 v = G2[i * BLK_MAX + c];
                for (int l = 0; l < i; ++l) v = csub(v, cjmul(R[l * BLK_MAX + i], R[l * BLK_MAX + c]));
                R[i * BLK_MAX + c] = cscale(v, 1.0 / rii);
            }
        }
        if (fi >= 0) {
            // the dependent vector z_{fi+1}: keep its coordinates on q_1..q_fi
            for (int c = fi; c < sb; ++c)
                for (int l = fi; l < BLK_MAX; ++l) R[l * BLK_MAX + c] = mk(0, 0);
            if (a.brk[b] < 0) a.brk[b] = j + fi;
        }
        const int nq = fi >= 0 ? fi : sb;
        // inverse of the leading nq x nq upper triangle
        for (int c = 0; c < nq; ++c) {
            Ri[c * BLK_MAX + c] = cdiv(mk(1, 0), R[c * BLK_MAX + c]);
            for (int r = c - 1; r >= 0; --r) {
                double2 v = mk(0, 0);
                for (int l = r + 1; l <= c; ++l) v = cadd(v, cmul(R[r * BLK_MAX + l], Ri[l * BLK_MAX + c]));
                Ri[r * BLK_MAX + c] = cscale(cdiv(v, R[r * BLK_MAX + r]), -1.0);
            }
        }
        sh_fi = fi;
    }
    __syncthreads();
    const int fi = sh_fi;
    const int nq = fi >= 0 ? fi : sb;           // new orthonormal columns
    const int bs = fi >= 0 ? fi + 1 : sb;       // H columns produced by this block
    // final update: q_o = sum_a x_a Ri[a][o] - sum_c v_c (Pc Ri)[c][o]
    for (int t = lane; t < BLK_MAX * BLK_MAX; t += 64) {
        const int o = t / BLK_MAX, q = t % BLK_MAX;
        beta[t] = (o < nq && q < nq) ? Ri[q * BLK_MAX + o] : mk(0, 0);
    }
    for (int t = lane; t < (j + 1) * BLK_MAX; t += 64) {
        const int c = t / BLK_MAX, o = t % BLK_MAX;
        double2 v = mk(0, 0);
        if (o < nq)
            for (int q = 0; q <= o; ++q) v = cadd(v, cmul(Pc[c * BLK_MAX + q], Ri[q * BLK_MAX + o]));
        coef[o * (MAXM + 1) + c] = v;
    }
    // H columns j..j+bs-1 (rows 0..m), by rows across the lanes
    double2* H = a.H + b * a.h_ms;
    const double2 th = a.thetas ? a.thetas[b] : a.theta;
    const double rho = a.rhos ? a.rhos[b] : a.rho;
    for (int r = lane; r <= a.m; r += 64) {
        // (H_old M_a)[r][c] over all columns l < j, for every c of the block
        // at once (each entry of row r read once; each sum still runs over l
        // in order): after a deflated restart the leading (k+1) x k block of
        // H_old is full, not Hessenberg
        double2 hmv[BLK_MAX];
#pragma unroll
        for (int c = 0; c < BLK_MAX; ++c) hmv[c] = mk(0, 0);
        if (r <= j)
            for (int l = 0; l < j; ++l) {
                const double2 h = H[(int64_t)l * a.ldh + r];
#pragma unroll
                for (int c = 1; c < BLK_MAX; ++c)
                    if (c < bs) hmv[c] = cadd(hmv[c], cmul(h, Ch[l * BLK_MAX + c - 1]));
            }
        double2 X[BLK_MAX];
#pragma unroll
        for (int c = 0; c < BLK_MAX; ++c) {
            if (c >= bs) break;
            // coordinates of z_{c+1} (Zc) and of z_c (Zh) on row r
            auto zc = [&](int cc) -> double2 {
                if (r <= j) return Ch[r * BLK_MAX + cc];
                const int l = r - j - 1;
                return (l <= cc && l < BLK_MAX) ? R[l * BLK_MAX + cc] : mk(0, 0);
            };
            const double2 zh = c == 0 ? mk(r == j ? 1.0 : 0.0, 0) : zc(c - 1);
            double2 t = cadd(cscale(zc(c), rho), cmul(th, zh));
            if (c >= 1 && r <= j) t = csub(t, hmv[c]);
            // X[:, c] = (T[:, c] - sum_{l<c} X[:, l] Mb[l][c]) / Mb[c][c]
            for (int l = 0; l < c; ++l) {
                const double2 mb = l == 0 ? Ch[j * BLK_MAX + c - 1] : R[(l - 1) * BLK_MAX + c - 1];
                t = csub(t, cmul(X[l], mb));
            }
            X[c] = c == 0 ? t : cdiv(t, R[(c - 1) * BLK_MAX + c - 1]);
        }
#pragma unroll
        for (int c = 0; c < BLK_MAX; ++c)
            if (c < bs) H[(int64_t)(j + c) * a.ldh + r] = r <= j + c + 1 ? X[c] : mk(0, 0);
    }
}

void sstep_small(const SstepArgs& a, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_sstep_small, dim3(nmem), dim3(64), 0, st, a);
}

void cycle_small(const CycleArgs& a, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_cycle_small, dim3(a.restart == 2 ? 1 : a.ns, nmem), dim3(64), 0, st, a);
}

// ---------------------------------------------------------------------------
// One block per (shift, member): every block solves the base problem (the
// shifted ones need d1 and y), block 0 stores it, block i >= 1 the system of
// shift i, so the shifts' QR factorisations run side by side.
__global__ __launch_bounds__(64) void k_proj_small(ProjArgs a) {
    const int lane = threadIdx.x;
    const int role = blockIdx.x;
    const int b = blockIdx.y;
    if (a.act && !a.act[b]) return;
    const int k = a.k;
    const int kp = a.kp;   // leading columns used (k: the full projection)
    const int ns = a.ns;
    const int ldk = k + 1;
    const double2* C = a.C + b * a.c_ms;
    const double2* sig = a.sigma + b * a.sig_ms;
    const double2* beta = a.beta + b * a.beta_ms;
    double2* gam = a.gam + b * a.gam_ms;
    double2* coef = a.coef + b * a.coef_ms;
    __shared__ double2 A[(MAXM + 2) * LD];
    __shared__ double2 hv[LD + 1], d1[LD + 1], y[LD + 1], di[LD + 1];
    const double2 s1 = sig[0];
    // [Hk(:, 0..kp-1) - sigma_1 I_bar | C]
    for (int c = 0; c <= kp; ++c)
        for (int r = lane; r <= k; r += 64) {
            double2 v = c < kp ? a.Hk[c * ldk + r] : C[r];
            if (c < kp && r == c) v = csub(v, s1);
            AT(A, r, c) = v;
        }
    __syncthreads();
    hh_qr(A, k + 1, kp, kp + 1, hv, k + 1);
    for (int r = lane; r < kp; r += 64) d1[r] = AT(A, r, kp);
    __syncthreads();
    bool bad = !back_sub(A, kp, d1);
    // y = (Hk(:, 0..kp-1) - sigma_1 I_bar) d1
    for (int r = lane; r <= k; r += 64) {
        double2 acc = mk(0, 0);
        for (int c = 0; c < kp; ++c) {
            double2 h = a.Hk[c * ldk + r];
            if (r == c) h = csub(h, s1);
            acc = cadd(acc, cmul(h, d1[c]));
        }
        y[r] = acc;
    }
    __syncthreads();
    if (role == 0)
        for (int r = lane; r <= k; r += 64) {
            coef[r] = r < kp ? d1[r] : mk(0, 0);
            coef[ns * (k + 1) + r] = mk(-y[r].x, -y[r].y);
        }
    if (role >= 1 && role < ns) {
        const int i = role;
        const double2 si = sig[i], bi = beta[i];
        __syncthreads();
        // first kp rows: (H - sigma_i I) d_i = beta_i (H - sigma_1 I) d_1
        for (int c = 0; c <= kp; ++c)
            for (int r = lane; r < kp; r += 64) {
                double2 v;
                if (c < kp) {
                    v = a.Hk[c * ldk + r];
                    if (r == c) v = csub(v, si);
                } else {
                    v = cmul(bi, y[r]);
                }
                AT(A, r, c) = v;
            }
        __syncthreads();
        hh_qr(A, kp, kp, kp + 1, hv, kp);
        for (int r = lane; r < kp; r += 64) di[r] = AT(A, r, kp);
        __syncthreads();
        if (!back_sub(A, kp, di)) bad = true;
        for (int r = lane; r <= k; r += 64) coef[i * (k + 1) + r] = r < kp ? di[r] : mk(0, 0);
        if (kp == k) {
            // gamma_i += h_{k+1,:} (beta_i d1 - d_i): the v_{k+1} component (eq. (4.1))
            double2 g = mk(0, 0);
            for (int c = lane; c < k; c += 64)
                g = cadd(g, cmul(a.Hk[c * ldk + k], csub(cmul(bi, d1[c]), di[c])));
            g = mk(wred(g.x), wred(g.y));
            if (lane == 0) gam[i] = cadd(gam[i], g);
        }
    }
    if (lane == 0 && bad) atomicOr(&a.flags[b], 1);
}

void proj_small(const ProjArgs& a, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_proj_small, dim3(a.ns, nmem), dim3(64), 0, st, a);
}


// ---------------------------------------------------------------------------
// Related right-hand sides (Sec. 5, eq. (5.2)): the shift-independent normal
// equations (B^H B) d = B^H b of the minres projection over earlier
// right-hand sides, one wavefront per member. G: np x np column-major (ld np)
// shared by all members; rhs: member b's B^H b at rhs + b*rhs_ms. Gaussian
// elimination with partial pivoting in LDS (lane = row). Output d at
// dout + b*d_ms and -d at dneg + b*d_ms; a numerically singular G (pivot
// below 1e-13 of the largest entry) gives d = 0, i.e. no projection.
__global__ __launch_bounds__(64) void k_gram_solve(const double2* __restrict__ G, int np,
                                                   const double2* __restrict__ rhs, int64_t rhs_ms,
                                                   double2* __restrict__ dout,
                                                   double2* __restrict__ dneg, int64_t d_ms) {
    const int lane = threadIdx.x;
    const int b = blockIdx.x;
    __shared__ double2 A[(MAXM + 2) * LD];
    __shared__ double2 x[LD + 1];
    __shared__ int piv;
    __shared__ int bad;
    double gmax = 0;
    for (int c = 0; c <= np; ++c)
        for (int r = lane; r < np; r += 64) {
            const double2 v = c < np ? G[(int64_t)c * np + r] : rhs[b * rhs_ms + r];
            AT(A, r, c) = v;
            if (c < np) gmax = fmax(gmax, cabs(v));
        }
    for (int o = 32; o >= 1; o >>= 1) gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
    if (lane == 0) bad = 0;
    __syncthreads();
    for (int k = 0; k < np; ++k) {
        if (lane == 0) {
            int p = k;
            double best = cabs(AT(A, k, k));
            for (int r = k + 1; r < np; ++r) {
                const double v = cabs(AT(A, r, k));
                if (v > best) {
                    best = v;
                    p = r;
                }
            }
            piv = p;
            if (!(best > 1e-13 * gmax)) bad = 1;
        }
        __syncthreads();
        if (bad) break;
        const int p = piv;
        if (p != k)
            for (int c = lane; c <= np; c += 64) {
                const double2 t = AT(A, k, c);
                AT(A, k, c) = AT(A, p, c);
                AT(A, p, c) = t;
            }
        __syncthreads();
        const double2 pv = AT(A, k, k);
        for (int r = k + 1 + lane; r < np; r += 64) {
            const double2 f = cdiv(AT(A, r, k), pv);
            for (int c = k + 1; c <= np; ++c) AT(A, r, c) = csub(AT(A, r, c), cmul(f, AT(A, k, c)));
        }
        __syncthreads();
    }
    if (!bad && lane == 0) {
        for (int r = np - 1; r >= 0; --r) {
            double2 acc = AT(A, r, np);
            for (int c = r + 1; c < np; ++c) acc = csub(acc, cmul(AT(A, r, c), x[c]));
            x[r] = cdiv(acc, AT(A, r, r));
        }
    }
    __syncthreads();
    for (int r = lane; r < np; r += 64) {
        const double2 v = bad ? mk(0, 0) : x[r];
        dout[b * d_ms + r] = v;
        dneg[b * d_ms + r] = mk(-v.x, -v.y);
    }
}

void gram_solve(const double2* G, int np, const double2* rhs, int64_t rhs_ms, double2* dout,
                double2* dneg, int64_t d_ms, int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_gram_solve, dim3(nmem), dim3(64), 0, st, G, np, rhs, rhs_ms, dout, dneg,
                       d_ms);
}

}  // namespace gdr
