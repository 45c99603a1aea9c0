/*
 * gdr.h -- C-ABI of the MI355X library for deflated, restarted GMRES on
 * multiply shifted systems with multiple right-hand sides:
 *
 *     (A - sigma_i I) x_i^j = b^j,   i = 1..ns (shifts), j = 1..nrhs,
 *
 * (Darnell, Morgan, Wilcox; Sec. 1, eq. (1.1)), with A the Wilson-Dirac
 * matrix A = I - kappa D of Sec. 4, Example 7. sigma_1 is the base shift.
 * There is no preconditioning (Sec. 1): all shifts share one Krylov space.
 *
 *  - the first right-hand side is solved by GMRES-DR-Sh (Sec. 3, algorithm
 *    GMRES-DR-Sh), which also produces the deflation pair
 *    A V_k = V_{k+1} H_bar_k (Sec. 2.2, eq. (2.9));
 *  - the extra right-hand side v_{k+1} and every later right-hand side are
 *    solved by GMRES-Proj-Sh (Sec. 4, the two GMRES-Proj-Sh algorithms),
 *    followed by the correction x_i += (v_{k+1}^H r_i) s_i (eqs. (4.3)-(4.6)).
 *
 * Conventions
 *  - Complex numbers are gdr_c64 {re, im} (binary compatible with C99
 *    double complex / numpy complex128).
 *  - Vectors cross the boundary in the canonical layout
 *    [t][z][y][x][spin 4][colour 3], complex128, n = 12*Lx*Ly*Lz*Lt, and
 *    several vectors are stored one after the other. All vector pointers are
 *    DEVICE pointers on the context's device unless stated otherwise.
 *  - Links: [mu = x,y,z,t][t][z][y][x][a 3][b 3] complex128, row-major 3x3,
 *    U_mu(x) multiplies psi(x + mu). No boundary phases folded in.
 *  - D psi(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *               + (1 + gamma_mu) U_mu(x-mu)^H psi(x-mu)
 *    in the chiral basis (gamma5 = diag(1,1,-1,-1)); a hop that wraps in
 *    direction mu is multiplied by bc[mu].
 *  - Every call is synchronous on return: work is ordered on the context's
 *    HIP stream and the call waits for it. No caller pointer is retained.
 *  - Return codes: GDR_OK (0), GDR_NOT_CONVERGED (1, outputs valid and
 *    residuals filled), or a negative error; gdr_last_error() describes it.
 *    A solve returns GDR_OK only if every final FP64 true residual
 *    ||b - (A - sigma_i) x_i|| / ||b|| is at most tol (plain FP64 checks them
 *    after the solve; mixed precision in its cleanup). In plain FP64 the
 *    corrected non-base shifts of later right-hand sides are only as accurate
 *    as the extra right-hand side's tolerance (Sec. 4) and can end above tol.
 *  - One context per host thread; calls on one context must not overlap.
 */
#ifndef GDR_H
#define GDR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } gdr_c64;
typedef struct gdr_ctx_s* gdr_ctx;
typedef struct gdr_op_s* gdr_op;
typedef struct gdr_defl_s* gdr_defl;

#define GDR_OK 0
#define GDR_NOT_CONVERGED 1
#define GDR_ERR_ARG (-1)       /* invalid argument (sizes, null pointers, m <= k, ...) */
#define GDR_ERR_HIP (-2)       /* a HIP runtime call failed */
#define GDR_ERR_OOM (-3)       /* device allocation failed */
#define GDR_ERR_BREAKDOWN (-4) /* singular small system: (Q^H s)_{m+1} = 0, 1 - gamma_i = 0,
                                  or H_k - sigma_i I singular (Secs. 2.1, 4) */
#define GDR_ERR_STATE (-5)     /* handle used inconsistently (wrong op, shift list mismatch) */

/* arithmetic of a solve or an operator application */
#define GDR_PREC_F64 0   /* everything in FP64 */
#define GDR_PREC_MIXED 1 /* FP32 matvecs, Gram-Schmidt and basis; FP64 small problems,
                            solution accumulation and true residuals (refinement) */
#define GDR_PREC_F32 1   /* gdr_op_apply only: FP32 arithmetic */

/* storage of the gauge links used by the FP32 operator */
#define GDR_LINKS_F64 0
#define GDR_LINKS_F32 1
#define GDR_LINKS_F16 2

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`; all work is queued on
 * `hip_stream` (a hipStream_t, or NULL for the default stream). The library
 * owns *out until gdr_ctx_destroy. Errors: ARG (null out, bad device), HIP. */
int gdr_ctx_create(int device, void* hip_stream, gdr_ctx* out);
void gdr_ctx_destroy(gdr_ctx ctx);
/* Last error message of the context (static storage owned by the context). */
const char* gdr_last_error(gdr_ctx ctx);

/* --------------------------------------------------------------- operator */

/* The Wilson-Dirac matrix A = I - kappa D (Sec. 4, Example 7) on an
 * Lx x Ly x Lz x Lt lattice, dims = {Lx, Ly, Lz, Lt}, every extent even and
 * >= 2. bc[mu] is +1 (periodic) or -1 (antiperiodic). `links` is host memory
 * (links_on_device = 0) or device memory (1) in the canonical link layout;
 * it is copied into internal tile-blocked layouts (FP64 always, plus FP32
 * or FP16 per link_storage for the FP32 operator; with FP16 storage also an
 * FP32 copy, which the refinement solves of the mixed-precision cleanup use)
 * and not retained. Special unitary links (to 1e-9) on lattices whose
 * extents are multiples of 4 are kept, in FP32 or FP16, as their first two
 * rows (gdr_op_link_bytes).
 * Errors: ARG, OOM, HIP. */
int gdr_wilson_create(gdr_ctx ctx, const int dims[4], const int bc[4], double kappa,
                      const gdr_c64* links, int links_on_device, int link_storage,
                      gdr_op* out);
void gdr_op_destroy(gdr_op op);

/* The bidiagonal test matrix of Examples 1-6 (Sec. 2.1, Sec. 3, Sec. 4) as an
 * operator for the same solvers: M has diagonal diag[0..n-1] and
 * superdiagonal super[0..n-2] (Example 1: diag = 0.1, 1, 2, ..., n-1 and
 * super = 1), host arrays, copied (FP64 plus an FP32 copy for mixed
 * precision) and not retained; the solvers then solve (M - sigma_i I) x = b.
 * Vectors are plain complex arrays of n entries. gdr_op_tables and the
 * lattice-only parts do not apply. Errors: ARG (n < 1, null or non-finite
 * entries), OOM, HIP. */
int gdr_bidiag_create(gdr_ctx ctx, int64_t n, const gdr_c64* diag, const gdr_c64* super,
                      gdr_op* out);
/* Number of complex unknowns n (12 * volume for the Wilson operator). */
int64_t gdr_op_size(gdr_op op);

/* Bytes of link storage per lattice site that one application of the
 * operator reads at `precision` (GDR_PREC_F64: 576; GDR_PREC_F32: 288 for
 * FP32 links, 144 for FP16-stored links, 192 (FP32) or 96 (FP16) when the
 * links are special unitary and stored as their first two rows, the third
 * being rebuilt as the conjugated cross product of the two - chosen by
 * gdr_wilson_create on lattices whose extents are multiples of 4). -1 for a
 * non-lattice operator or an unknown precision. */
int gdr_op_link_bytes(gdr_op op, int precision);

/* y_v = (A - sigma I) x_v for v = 0..nvec-1 (eq. (1.1)), canonical layout,
 * device pointers, x and y each nvec*n complex128 (must not overlap).
 * precision GDR_PREC_F64 or GDR_PREC_F32 (FP32 arithmetic with the op's
 * link storage; input rounded to FP32, output widened). Errors: ARG, HIP. */
int gdr_op_apply(gdr_op op, gdr_c64 sigma, const gdr_c64* x, gdr_c64* y, int nvec,
                 int precision);

/* gdr_op_apply without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same y_v = (A - sigma I) x_v, same
 * layouts and arguments. Its internal-layout staging buffers live in one
 * static 64 MiB device array per GPU (held until the process ends), so n is
 * limited to 2^21 unknowns in FP64 (2^22 in FP32) - larger operators return
 * GDR_ERR_ARG; more vectors than fit run in chunks. Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (from several
 * threads or contexts) race and must be serialised by the caller. Nothing in
 * the array needs to start cleared (each chunk is written before it is
 * read). Errors: ARG, HIP. */
int gdr_op_apply_noalloc(gdr_op op, gdr_c64 sigma, const gdr_c64* x, gdr_c64* y, int nvec,
                         int precision);

/* Test hook: the even-odd index of every lexicographic site
 * (eo = parity*V/2 + lex/2, lex = x + Lx(y + Ly(z + Lz t))), the neighbour
 * table nbr[eo][d] in even-odd positions for hops d = +x,+y,+z,+t,-x,-y,-z,-t
 * and sign[eo][d] = -1 where the hop crosses the time boundary. Host buffers
 * of V, 8V and 8V entries, computed on the device. Errors: ARG, HIP. */
int gdr_op_tables(gdr_op op, int32_t* eo_of_lex, int32_t* nbr, int8_t* sign);

/* Measurement hook for the operator alone (the matrix-vector product of
 * Sec. 4, Example 7): `reps` launches of y = (A - sigma I) x on nvec vectors
 * held in the library's internal layout, rotating over `nsets` separate
 * input/output buffer sets (allocated and filled by the library, so that the
 * 256 MB Infinity Cache cannot keep one set resident), each launch timed with
 * HIP events on the context stream. precision GDR_PREC_F64 (FP64 vectors and
 * links) or GDR_PREC_F32 (FP32 vectors, the op's FP32 or FP16 links).
 * ms_each: caller host array of `reps` entries (per-launch milliseconds).
 * 1 <= nvec <= 16, 1 <= nsets <= 8, 1 <= reps <= 100000.
 * Errors: ARG, OOM, HIP. */
int gdr_op_dslash_bench(gdr_op op, int precision, int nvec, int nsets, int reps,
                        double* ms_each);

/* ------------------------------------------------------------ parameters */

typedef struct {
    int m_dr;          /* GMRES-DR(m, k) subspace size for the first RHS (Sec. 2.2), m <= 64 */
    int k;             /* number of deflated harmonic Ritz vectors, 0 <= k < m_dr */
    int m_proj;        /* GMRES(m)-Proj(k) cycle length for later RHS (Sec. 2.3), k < m_proj <= 64 */
    double tol;        /* relative residual ||b - (A - sigma_i) x_i|| / ||b|| per (shift, RHS) */
    double tol_extra;  /* tolerance of the extra right-hand side v_{k+1} (Sec. 4, Example 6);
                          <= 0 selects sqrt(tol) */
    int max_cycles;    /* cap on restart cycles per phase */
    int precision;     /* GDR_PREC_F64 or GDR_PREC_MIXED */
    int batch;         /* 1: later RHS run as one batch (one matvec launch per step) */
    int related_rhs;   /* 1: project over earlier solutions first (Sec. 5, eq. (5.2)) */
    int max_refine;    /* mixed precision: cap on refinement rounds of the cleanup */
    int profile;       /* bitmask of GDR_K_* kernel classes to time with HIP events on the
                          context stream (0: none); results in gdr_stats.k_* */
    int m_clean;       /* cycle length of the mixed-precision cleanup solves (0: automatic) */
    int proj_k;        /* 0: later RHS project over all k deflation vectors with the v_{k+1}
                          component tracked, the extra RHS and the correction (Sec. 4);
                          1..k: project over the leading proj_k (most accurate) approximate
                          eigenvectors only, no extra RHS and no correction (Sec. 4,
                          Theorem 1 and Table 4.1) */
    int use_graph;     /* 1: each Arnoldi cycle is captured once into a HIP graph and replayed
                          (fewer launches for small lattices; ignored while profiling) */
    int galerkin;      /* 0: the deflated first-RHS phase is GMRES-DR-Sh (minimum residual
                          base system, Sec. 3); 1: FOM-DR-Sh instead (Galerkin condition for
                          every shift, residuals parallel by construction, Ritz deflation;
                          Sec. 3, Examples 2 and 3), and with k = 0 FOM(m)-Sh. Later RHS
                          keep GMRES-Proj-Sh. A singular Galerkin system returns
                          GDR_ERR_BREAKDOWN. */
    int sstep;         /* FP32 Arnoldi of the mixed path: 0 or 1 one vector per step (delayed
                          classical Gram-Schmidt twice, two sweeps over the basis per step);
                          2..8 blocks of sstep vectors (powers of (A - c)/r on a disc holding
                          the spectrum, block Gram-Schmidt with a Cholesky factor: two sweeps
                          per block, four when the second pair runs; blocks of 5..8 take the
                          FP64 matrix-core sweeps and need an operator size divisible by 16,
                          else blocks of 4 are used). Same Krylov space and Arnoldi relation;
                          the FP64 path always takes one vector per step. */
    double sstep_reorth; /* s-step blocks: one projection and one update sweep per block unless
                          the projection removed more than this ratio of a block vector's norm
                          squared (its FP32 rounding would then leave components along the
                          basis): then a second pair. 0: always two pairs. Default 20. */
    double refine_floor; /* mixed precision: each refinement round of the cleanup solves the
                          residual system in FP32 to relative tolerance max(0.3 tol / res,
                          refine_floor). 0: 1e-5. Must be in [0, 0.5]. */
    int persistent;    /* gdr_solve_many only: 1 runs the first right-hand sides of all its
                          lattices as one batch with persistent work-list operator launches
                          (see there); 0 solves the lattices one after another. 0 or 1. */
} gdr_params;

/* kernel classes of the profiler (gdr_params.profile bit i = class i) */
#define GDR_K_DSLASH 0      /* Wilson operator launches of the Krylov space (FP32 in the mixed path,
                               FP64 in the FP64 path) */
#define GDR_K_GS_PROJECT 1  /* Gram-Schmidt projection sweep V^H [r_j, A r_j] */
#define GDR_K_GS_UPDATE 2   /* Gram-Schmidt update sweep (finishes q_j, forms r_{j+1}) */
#define GDR_K_GS_CLOSE 3    /* second Gram-Schmidt passes: the closing pass of the last basis
                               column (one vector per step), or the second block sweep pair of the
                               s-step cycle, masked per member on the device (no bytes counted) */
#define GDR_K_SMALL 4       /* device small dense problems */
#define GDR_K_COMBINE 5     /* x_i += V d_i, r = V s */
#define GDR_K_RECOMBINE 6   /* V_{k+1} = V_{m+1} P */
#define GDR_K_OTHER 7       /* FP64 true residuals of the mixed path, reductions, scaling */

/* Fill defaults: m_dr 40, k 15, m_proj 40, tol 1e-8, tol_extra sqrt(tol),
 * max_cycles 1000, FP64, batch 1, related 0, max_refine 8, profile 0, m_clean 0,
 * proj_k 0, use_graph 0, galerkin 0, sstep 8, sstep_reorth 20, refine_floor 0,
 * persistent 0. */
void gdr_params_default(gdr_params* p);

typedef struct {
    int cycles_dr, cycles_extra, cycles_proj, cycles_cleanup;
    int64_t mvp_dr;      /* operator applications of the GMRES-DR-Sh phase */
    int64_t mvp_extra;   /* ... of the extra right-hand side */
    int64_t mvp_proj;    /* ... of the later right-hand sides (sum over RHS) */
    int64_t mvp_fp64;    /* FP64 true-residual applications (correction, replacement, checks) */
    int64_t mvp_cleanup; /* ... of the mixed-precision cleanup solves */
    double t_total;      /* seconds */
    double t_phase[8];   /* seconds: 0 DR, 1 extra, 2 proj, 3 correction, 4 cleanup, 5 verify */
    double* resid;       /* caller host array [nrhs][ns] or NULL: true FP64 relative residuals */
    double* hist;        /* caller host array [hist_cap][5] or NULL: per cycle
                            (phase, cycle, mvps, ||r_1||/||b||, max_i |beta_i| ||r_1||/||b||);
                            phase 0 DR, 1 extra, 2+j later RHS j (max over the batch) */
    int hist_cap, hist_len;
    gdr_c64* theta;      /* caller host array [theta_cap] or NULL: the k harmonic Ritz values
                            kept at every GMRES-DR restart, in selection order */
    int theta_cap, theta_len;
    double k_ms[8];      /* per kernel class (GDR_K_*) timed with params.profile: total ms */
    double k_bytes[8];   /* ... algorithmic HBM bytes of those launches (each operand once) */
    double k_flops[8];   /* ... algorithmic flops */
    int64_t k_launches[8];
    double resid_main;   /* mixed precision: largest true relative residual before the cleanup */
} gdr_stats;

/* ---------------------------------------------------------------- solvers */

/* First right-hand side by GMRES-DR(m_dr, k)-Sh (Sec. 3). sigma: host array
 * of ns shifts, sigma[0] the base (should be the slowest to converge,
 * Sec. 3, Example 3). b: device n-vector. x: device ns*n output (zero
 * initial guess, Sec. 5). If defl_out is not NULL it receives the deflation
 * pair (V_{k+1}, H_bar_k) (eq. (2.9)), owned by the caller until
 * gdr_defl_destroy. Errors: ARG, OOM, HIP, BREAKDOWN; NOT_CONVERGED. */
int gdr_solve_dr_sh(gdr_op op, int ns, const gdr_c64* sigma, const gdr_c64* b, gdr_c64* x,
                    const gdr_params* p, gdr_stats* st, gdr_defl* defl_out);

/* Right-hand sides B (device, nrhs*n) by GMRES(m_proj)-Proj(k)-Sh with the
 * correction (Sec. 4). X: device nrhs*ns*n output. On first use with a
 * shift list the extra right-hand side v_{k+1} is solved and its solutions
 * s_i cached in defl; a different shift list recomputes them.
 * Errors: ARG, STATE (defl from another operator), OOM, HIP, BREAKDOWN. */
int gdr_solve_proj_sh(gdr_op op, gdr_defl defl, int ns, const gdr_c64* sigma, int nrhs,
                      const gdr_c64* B, gdr_c64* X, const gdr_params* p, gdr_stats* st);

/* Whole problem in the paper's order of use (Sec. 4): RHS 0 by GMRES-DR-Sh,
 * then the extra RHS, then RHS 1..nrhs-1 by GMRES-Proj-Sh and correction;
 * mixed precision adds an FP64-refined cleanup. X: device nrhs*ns*n. */
int gdr_solve(gdr_op op, int ns, const gdr_c64* sigma, int nrhs, const gdr_c64* B,
              gdr_c64* X, const gdr_params* p, gdr_stats* st);

/* ------------------------------------------------------- deflation handle */

/* Independent problems on several lattices (Sec. 1, eq. (1.1) for each
 * operator): (A_l - sigma_i I) x_i^{l,j} = b^{l,j}, l < nops, with the same
 * ns shifts, nrhs right-hand sides and parameters for every lattice, each
 * solved as gdr_solve solves it. B[l] (device, nrhs x n_l canonical
 * complex128, n_l = gdr_op_size(ops[l])) and X[l] (device, nrhs x ns x n_l)
 * belong to ops[l]'s context; st is NULL or an array of nops records, one per
 * lattice. params->persistent = 0: the lattices one after another, each on
 * its own context. params->persistent = 1 (mixed precision with s-step blocks,
 * at most 16 Wilson operators whose links are stored as two rows in one
 * precision, lattices of any sizes with extents multiples of 4, all on one
 * device): GMRES-DR-Sh on the first right-hand sides runs for all lattices as
 * one batch, on the first operator's context: every operator application is
 * one persistent work-list launch over the tiles of all lattices, every
 * Gram-Schmidt sweep and combination one launch over the lattices, each
 * lattice keeping its own Krylov space, restarts and stopping rule. The
 * extra right-hand side, the later right-hand sides and the cleanup then run
 * per lattice on the lattice's own context, concurrently in host threads for
 * lattices on different contexts. Returns GDR_OK when every lattice's solve
 * does, else the first other status; errors (reported on the first
 * operator's context): ARG (requirements, arguments), OOM, HIP, BREAKDOWN. */
int gdr_solve_many(int nops, const gdr_op* ops, int ns, const gdr_c64* sigma, int nrhs,
                   const gdr_c64* const* B, gdr_c64* const* X, const gdr_params* params,
                   gdr_stats* st);

/* Number k of deflation vectors (V holds k+1 columns). */
int gdr_defl_k(gdr_defl d);
/* Copy out V_{k+1} (device, (k+1)*n canonical complex128) and H_bar_k (host,
 * (k+1) x k, column-major complex128); either pointer may be NULL. */
int gdr_defl_export(gdr_defl d, gdr_c64* V, gdr_c64* Hbar);
/* Build a handle from an exported pair (same layouts) for operator op;
 * precision selects the basis storage (F64 or MIXED = FP32). */
int gdr_defl_import(gdr_op op, int k, const gdr_c64* V, const gdr_c64* Hbar, int precision,
                    gdr_defl* out);
void gdr_defl_destroy(gdr_defl d);

/* ---- Launch tuning --------------------------------------------------------
 * Some launches have several equivalent forms (tile order and kernel variant
 * of the Wilson operator, strips per wavefront of the restart recombination
 * V_{k+1} = V_{m+1} P of Sec. 2.2, blocks per member of the Gram-Schmidt
 * update sweeps and of the solution accumulation): each computes every output
 * with the same operations in the same order, so the choice never changes a
 * result. The first launches of a (kernel, shape) on a device time the forms
 * in turn with HIP events; after 3 timings each the fastest is kept for the
 * process. Environment: GDR_TUNE=0 keeps the default forms; GDR_TUNE_CACHE
 * names a text file read at the first launch and appended to at each decision
 * (one line "v1 <kernel>|<arch>|<shape> <form> <median us per unit of work>";
 * malformed lines are skipped, an absent file is not an error). While forms
 * are still timed, Arnoldi cycles run eagerly instead of from a HIP graph
 * (at most four cycles per solve). Process-wide; thread-safe. */
/* Read decisions from a cache file in the format above (on top of those read
 * from GDR_TUNE_CACHE). Returns the number of lines taken, GDR_ERR_ARG for a
 * NULL path or a file that cannot be opened. */
int gdr_tune_load(const char* path);
/* The decisions taken so far, one "<kernel>|<arch>|<shape> -> <form> (<us> us
 * per unit)" line each, NUL-terminated into buf (host, len bytes, truncated
 * to fit; buf may be NULL when len is 0). Returns the full length without the
 * NUL, so a caller can size buf. */
int64_t gdr_tune_report(char* buf, int64_t len);

#ifdef __cplusplus
}
#endif
#endif /* GDR_H */
