// Small dense FP64 problems of every restart cycle, solved on the device by
// one 64-lane wavefront per problem with the matrices resident in LDS.
#pragma once

#include "common.h"

namespace gdr {

// Per-cycle results read back by the host (one small copy per cycle).
struct CycleOut {
    double snorm;               // ||s|| = ||r_1|| (shortcut norm, eq. (2.6))
    int flags;                  // bit0 singular shifted system, bit1 Schur failed
    int pad;
    double2 beta[MAXNS];        // beta_i^new
    double2 theta[MAXM];        // kept harmonic Ritz values (restart only)
    long long tclk[8];          // restart phase timestamps (wall_clock64 ticks)
};

struct CycleArgs {
    const double2* H;   // (m+1) x m column-major, ldh = m+1   (per member: + b*h_ms)
    int64_t h_ms;
    const double2* c;   // m+1                                (per member: + b*c_ms)
    int64_t c_ms;
    const double2* sigma;   // ns shifts                       (per member: + b*sig_ms)
    int64_t sig_ms;
    const double2* beta;    // ns current beta_i               (per member: + b*beta_ms)
    int64_t beta_ms;
    const int* brk;         // per member first breakdown step or -1
    double2* coef;          // (m+1) x (ns+1) column-major: d_i padded, last column s
    int64_t coef_ms;
    CycleOut* out;          // per member
    // 0: least squares only; 1: least squares and GMRES-DR restart (block 0);
    // 2: restart only (one block per member; s read from the coefficient block)
    int restart;
    int k;
    double2* P;             // (m+1) x (k+1), ldp = m+1              (per member: + b*p_ms)
    double2* Hnew;          // (m+1) x m zero except the leading (k+1) x k block (+ b*hnew_ms)
    double2* cnew;          // m+1                                   (per member: + b*cnew_ms)
    int64_t p_ms = 0, hnew_ms = 0, cnew_ms = 0;
    int m;
    int ns;
    const int* act;         // per member active flag (nullable)
    // 0: GMRES-Sh (base least squares, Ritz deflation by harmonic Ritz pairs);
    // 1: FOM-Sh (square Galerkin systems for every shift, Ritz pairs)
    int galerkin;
};

struct ProjArgs {
    const double2* Hk;      // (k+1) x k column-major (ld k+1)
    int k;
    int kp;                 // leading deflation vectors used, 1..k (k: full projection
                            // with the v_{k+1} component tracked in gam)
    const double2* C;       // per member k+1 coefficients V_{k+1}^H r (+ b*c_ms)
    int64_t c_ms;
    const double2* sigma;   // shifts of member b: sigma + b*sig_ms
    int64_t sig_ms;
    const double2* beta;    // per member ns
    int64_t beta_ms;
    double2* gam;           // per member ns (accumulated gamma_i)
    int64_t gam_ms;
    double2* coef;          // per member (k+1) x (ns+1): D padded with zero row, last column -y
    int64_t coef_ms;
    int* flags;             // per member: bit0 singular shifted k x k system
    int ns;
    const int* act;         // per member active flag (nullable)
};

// Small FP64 part of one block of the s-step Arnoldi cycle (one wavefront per
// member). The block starts from the orthonormal column j; Z = [z_1..z_sb]
// (columns j+1..j+sb) holds z_i = (A - theta) z_{i-1} / rho with z_0 = v_j.
// G holds the reduced sums [V_{0..j}, Z]^H Z of the sweep just made (value
// a*nc + c, nc = j+1+sb).
//   mode 1 (after the first projection): P1 = V_{0..j}^H Z, the raw norms
//     ||z_a||^2 and the Gram matrix Z^H Z - P1^H P1 of Z - V P1. If every
//     pivot keeps more than 1/reorth of its raw norm (reorth > 0), this sweep
//     suffices: as mode 2 with P2 = P1 and Z' = Z, reo[b] = 0. Otherwise the
//     coefficients of Z' = Z - V_{0..j} P1 and reo[b] = 1.
//   mode 2 (after the second projection, Z'; members with reo set): P2 =
//     V_{0..j}^H Z', the Cholesky factor R of Z'^H Z' - P2^H P2 (Z'' = Q R);
//     coefficients of Q = (Z' - V_{0..j} P2) R^{-1}; H columns j..j+sb-1 from
//     A Zhat = Z diag(rho) + Zhat diag(theta) in the basis [V_{0..j}, Q]
//     with C-hat = P1 + P2.
// A pivot below 1e-10 of the raw ||z_a||^2 is a breakdown (the Krylov space
// is invariant): brk = j + a, the later block vectors are zero.
struct SstepArgs {
    const double2* G;
    int64_t g_ms;
    int j, sb, mode, m;
    double2* Psave;   // per member (MAXM+1) x BLK_MAX, P1[c][a] at c*BLK_MAX + a
    int64_t p_ms;
    double* znorm;    // per member BLK_MAX
    double2* coef;    // per member BLK_COEF_MS
    int64_t coef_ms;
    double2* H;       // (m+1) x m column-major per member
    int64_t ldh, h_ms;
    double2 theta;
    double rho;
    const double2* thetas = nullptr;   // per member centre and radius (members on
    const double* rhos = nullptr;      //   different operators); else theta, rho
    int* brk;
    const int* act;
    double reorth;    // cancellation ratio above which a block gets a second sweep pair
    int* reo;         // per member: second sweep pair needed (mode 1 writes it)
};
void sstep_small(const SstepArgs& a, int nmem, hipStream_t st);

void cycle_small(const CycleArgs& a, int nmem, hipStream_t st);
void proj_small(const ProjArgs& a, int nmem, hipStream_t st);
// (B^H B) d = B^H b for related right-hand sides (np <= MAXM), d and -d per member
void gram_solve(const double2* G, int np, const double2* rhs, int64_t rhs_ms, double2* dout,
                double2* dneg, int64_t d_ms, int nmem, hipStream_t st);

}  // namespace gdr
