// Host-side launchers of the HIP kernels (all asynchronous on `st`).
#pragma once

#include "common.h"

namespace gdr {

// ------------------------------------------------------------ layout (layout.hip)
// canonical complex128 [v][t][z][y][x][4][3]  <->  internal tile-blocked SoA of
// type T, vector v at dst + v*stride (elements)
template <typename T>
void pack_spinor(const double2* canon, typename CT<T>::t* dst, int64_t stride, const Geom& g,
                 int nvec, hipStream_t st);
template <typename T>
void unpack_spinor(const typename CT<T>::t* src, int64_t stride, double2* canon, const Geom& g,
                   int nvec, hipStream_t st);
// storage: 0 FP64 (double2), 1 FP32 (float2), 2 FP16 (__half2 per complex),
// 3 FP32 rows 0 and 1 of special unitary links (LINK_R12; bc not folded),
// 4 the same rows in FP16 (LINK_R12H, __half2 per complex; bc not folded)
constexpr int LINK_R12 = 3;
constexpr int LINK_R12H = 4;
void pack_links(const double2* canon, void* out, int storage, const Geom& g, const int bc[4],
                hipStream_t st);
// largest deviation of nlinks canonical 3x3 links from SU(3) (see layout.hip);
// *dev_bits must be zeroed first, read it back as a double
void su3_deviation(const double2* canon, int64_t nlinks, unsigned long long* dev_bits,
                   hipStream_t st);
void build_tables(int32_t* eo_of_lex, int32_t* nbr, int8_t* sign, const Geom& g, int bc_t,
                  hipStream_t st);

// ------------------------------------------------------------ Dslash (dslash.hip)
constexpr int DSLASH_MAXV = 16;
struct DiagList {
    double2 d[DSLASH_MAXV];   // per-vector diagonal factor (1 - sigma_v)
    double alpha[DSLASH_MAXV];
};
// out_v = alpha_v * ((1 - sigma_v) in_v - kappa D in_v) [+ add_v]   for v < nvec
// TS spinor type; link storage per `link_storage`; compute in TS.
// anti: bit mu set when direction mu is antiperiodic (used with LINK_R12,
// whose links carry no boundary factor). Members with act[v] == 0 are skipped.
// Several lattices' operators in one persistent launch (FP32 spinors,
// two-row links): member v (v < nm <= DSLASH_MAXV) is a lattice of geometry
// g[v] (4^4 tiles) whose tiles are the work items tile0[v] .. tile0[v+1]-1.
struct LatList {
    int nm;
    int tile0[DSLASH_MAXV + 1];
    Geom g[DSLASH_MAXV];
    const void* links[DSLASH_MAXV];
    float kappa[DSLASH_MAXV];
    int anti[DSLASH_MAXV];
};
void dslash_list(const float2* in, int64_t in_stride, float2* out, int64_t out_stride,
                 const LatList& L, int link_storage, const DiagList& dl, hipStream_t st,
                 const int* act, int max_blocks);

template <typename TS>
void dslash(const typename CT<TS>::t* in, int64_t in_stride, typename CT<TS>::t* out,
            int64_t out_stride, const typename CT<TS>::t* add, int64_t add_stride,
            const void* links, int link_storage, const Geom& g, double kappa, const DiagList& dl,
            int nvec, hipStream_t st, const int* act = nullptr, int anti = 0);
// vectors per launch from which the FP32 LINK_R12 operator runs the vector-loop
// kernel (links held in registers across the vectors of one tile)
constexpr int DSLASH_VLOOP_MIN = 2;

// ------------------------------------------------------------ bidiagonal operator (bidiag.hip)
// out_v = alpha_v * (M in_v - sigma_v in_v) [+ add_v], sigma_v = 1 - dl.d[v];
// de: diagonal (n entries) then superdiagonal (n - 1 used), type T
template <typename T>
void bidiag_apply(const typename CT<T>::t* in, int64_t in_stride, typename CT<T>::t* out,
                  int64_t out_stride, const typename CT<T>::t* add, int64_t add_stride,
                  const typename CT<T>::t* de, int64_t n, const DiagList& dl, int nvec,
                  hipStream_t st, const int* act = nullptr);
// y_v = (TO) x_v for plain vectors
template <typename TI, typename TO>
void plain_copy(const typename CT<TI>::t* x, int64_t x_stride, typename CT<TO>::t* y,
                int64_t y_stride, int64_t n, int nvec, hipStream_t st);

// ------------------------------------------------------------ DCGS2 (blas.hip)
// Column-block sums of V_{0..nc-1}^H x_a (a < 1 or 2; x1 == nullptr for one
// vector) and ||x_last||^2 into partial[((mem*nval) + a*nc + c)*nblk + blk],
// nval = (#x)*nc + 1; reduce with reduce_cols(partial, nblk, nval, ...).
template <typename T, typename TX>
void gs_dot(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
            const typename CT<TX>::t* x0, int64_t x0_ms, const typename CT<TX>::t* x1,
            int64_t x1_ms, double2* partial, int nblk, int64_t n, int nmem, hipStream_t st,
            const int* act = nullptr);
// The same sums (one vector per member, nval = nc + 1) when every member
// projects on one shared basis V. An FP32 basis with FP64 members and n a
// multiple of 16 runs on the FP64 matrix cores, 16 members per block (the
// basis read once per 16 members; the sums in another order than gs_dot's);
// otherwise the VALU form reads the basis once per group of SHARED_MG members
// and gives gs_dot's partials bit for bit. Needs nc <= SHARED_NC_MAX; V is
// the same for all members (no member stride).
constexpr int SHARED_MG = 4;
constexpr int SHARED_NC_MAX = 32;
template <typename T, typename TX>
void shared_dot(const typename CT<T>::t* V, int64_t ldv, int nc, const typename CT<TX>::t* x,
                int64_t x_ms, double2* partial, int nblk, int64_t n, int nmem, hipStream_t st,
                const int* act = nullptr);
// y_o = sum_a beta[o][a] x_a - V_{0..nc-1} coef[o] (o < 1 or 2 outputs as inputs);
// layout of coef per member: coef[o*(MAXM+1) + c], beta at 2*(MAXM+1) + 2*o + a.
constexpr int GS_COEF_MS = 2 * (MAXM + 1) + 4;
template <typename T>
void gs_update(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
               const typename CT<T>::t* x0, int64_t x0_ms, const typename CT<T>::t* x1,
               int64_t x1_ms, typename CT<T>::t* y0, int64_t y0_ms, typename CT<T>::t* y1,
               int64_t y1_ms, const double2* coef, int64_t coef_ms, int64_t n, int nmem,
               hipStream_t st, const int* act = nullptr);
// Block Gram-Schmidt of the s-step Arnoldi cycle (block of nx <= BLK_MAX new
// vectors X_a = X + a*ldx, member b at + b*x_ms):
//   blk_dot:    partial sums of V_c^H X_a, c < nc, value a*nc + c (nval = nx*nc)
//   blk_update: in place, X_o <- sum_a X_a beta[o][a] - sum_{c<nc} V_c coef[o][c]
// with coef[o*(MAXM+1) + c] and beta[BLK_MAX*(MAXM+1) + o*BLK_MAX + a].
template <typename T>
void blk_dot(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
             const typename CT<T>::t* X, int64_t ldx, int64_t x_ms, int nx, double2* partial,
             int nblk, int64_t n, int nmem, hipStream_t st, const int* act = nullptr,
             bool second = false);
template <typename T>
void blk_update(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
                typename CT<T>::t* X, int64_t ldx, int64_t x_ms, int nx, const double2* coef,
                int64_t coef_ms, int64_t n, int nmem, hipStream_t st, const int* act = nullptr,
                bool second = false);
// DCGS2 bookkeeping of step j (see blas.hip): H corrections, next H column and
// the update coefficients, breakdown flag.
void dcgs_coef(const double2* G, int64_t g_ms, int j, int nx, int first, double2* H, int64_t ldh,
               int64_t h_ms, double2* coef, int64_t coef_ms, double* ref, int* brk, double tol,
               int nmem, hipStream_t st, const int* act = nullptr);

// ------------------------------------------------------------ BLAS (blas.hip)
// Block-partial buffers: partial[(member*ncols_tot + col)*nblk + blk] (double2);
// blocks per sweep over n rows
int cgs_nblk(int64_t n, int nmem = 1, bool wide = false);

// out[b*out_mstride + c] (+)= sum_blk partial[(b*ncols + c)*nblk + blk], c < ncols
void reduce_cols(const double2* partial, int nblk, int ncols, double2* out, int64_t out_mstride,
                 double2* add_to, int64_t add_mstride, int nmem, hipStream_t st,
                 const int* act = nullptr);

// out_s = beta_s * out_s + sum_{l<ncols} V_l * coef[l + s*ldc]   (FP64 outputs)
// member b: V + b*v_mstride, coef + b*c_mstride, out + b*o_mstride + s*o_stride.
// keep_mask bit s set: accumulate (beta 1); clear: overwrite (beta 0).
template <typename T>
void vcombine(const typename CT<T>::t* V, int64_t ldv, int64_t v_mstride, int ncols,
              const double2* coef, int ldc, int64_t c_mstride, int nout, double2* out,
              int64_t o_stride, int64_t o_mstride, unsigned keep_mask, int64_t n, int nmem,
              hipStream_t st, const int* act = nullptr);

// Basis recombination W_j = sum_{l<ncols} V_l P[l + j*ldp], j < nout, written as type T
template <typename T>
void vrecombine(const typename CT<T>::t* V, int64_t ldv, int ncols, const double2* P, int ldp,
                int nout, typename CT<T>::t* W, int64_t ldw, int64_t n, hipStream_t st);

// y_b = (T) (x_b * scal[b])  (scal device, may be null -> 1)  FP64 -> T conversion
template <typename T>
void convert_scale(const double2* x, int64_t x_mstride, const double* scal, int sc_stride,
                   typename CT<T>::t* y, int64_t y_mstride, int64_t n, int nmem, hipStream_t st,
                   const int* act = nullptr);

// x_b += coef[b*cstride] * y_b  (coef device double2; null -> 1)
void axpy_dev(double2* x, int64_t x_mstride, const double2* y, int64_t y_mstride,
              const double2* coef, int cstride, int64_t n, int nmem, hipStream_t st,
              const int* act = nullptr);
// start of a GMRES cycle per member: rn2[b*rs] = ||r||^2 ->
// c[b*cs + 0] = ||r||, c[b*cs + 1..m] = 0, inv[b] = 1/||r|| (0 if ||r|| = 0)
void start_cycle(const double2* rn2, int64_t rs, double2* c, int64_t cs, int m, double* inv,
                 int nmem, hipStream_t st, const int* act = nullptr);
// fill n ints with v
void fill_int(int* p, int v, int n, hipStream_t st);
// x_b *= coef[b]
void scal_dev(double2* x, int64_t x_mstride, const double2* coef, int64_t n, int nmem,
              hipStream_t st);
// y_b = x_b (double)
void copy_vec(const double2* x, int64_t x_mstride, double2* y, int64_t y_mstride, int64_t n,
              int nmem, hipStream_t st);

// ------------------------------------------------------------ small dense FP64 (small.hip)
struct SmallArgs;   // defined in small.h
}  // namespace gdr
