// Vector kernels of the Arnoldi recurrence (eq. (2.2)): classical Gram-Schmidt
// applied twice (CGS2) against the Krylov basis, norms, scaling, and the
// tall-skinny combinations x_i += V d_i, r = V s and V_{k+1} = V_{m+1} P.
//
// Dot products V^H w: each lane of a wavefront owns one row of a 64-row tile
// and forms the products of its row with 16 basis columns; a butterfly
// reduce-scatter over the wavefront (shuffles at distance 32,16,8,4, then an
// all-reduce over 2,1) leaves column (lane>>2)&15's tile sum on four lanes,
// which accumulate it over the wave's tiles in one register. Blocks write
// per-column partial sums; a second kernel adds them in a fixed order, so
// every result is bitwise reproducible. All accumulation is FP64.
#include "kernels.h"

namespace gdr {

__device__ __forceinline__ double2 shx(double2 v, int m) {
    return mk(__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64));
}

// reduce-scatter of 16 per-lane values over a 64-lane wavefront; returns the
// full sum of value (lane>>2)&15
__device__ __forceinline__ double2 rs16(const double2 (&a)[16], int lane) {
    double2 b[8], c[4], d[2];
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8, h2 = lane & 4;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        double2 send = h5 ? a[i] : a[i + 8];
        double2 keep = h5 ? a[i + 8] : a[i];
        b[i] = cadd(keep, shx(send, 32));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        double2 send = h4 ? b[i] : b[i + 4];
        double2 keep = h4 ? b[i + 4] : b[i];
        c[i] = cadd(keep, shx(send, 16));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        double2 send = h3 ? c[i] : c[i + 2];
        double2 keep = h3 ? c[i + 2] : c[i];
        d[i] = cadd(keep, shx(send, 8));
    }
    double2 e = cadd(h2 ? d[1] : d[0], shx(h2 ? d[0] : d[1], 4));
    e = cadd(e, shx(e, 2));
    e = cadd(e, shx(e, 1));
    return e;
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

int cgs_nblk(int64_t n) {
    int64_t tiles = (n + 63) / 64;
    int64_t nb = (tiles + 7) / 8;   // >= 2 tiles per wave on average
    if (nb > 1024) nb = 1024;
    if (nb < 1) nb = 1;
    return (int)nb;
}

template <typename T, typename TW, int MODE, bool CACHE>
__global__ __launch_bounds__(256) void k_cgs(const typename CT<T>::t* __restrict__ V, int64_t ldv,
                                             int64_t v_ms, int ncols,
                                             const typename CT<TW>::t* __restrict__ win,
                                             int64_t win_ms, double2* __restrict__ wd,
                                             int64_t wd_ms, const double2* __restrict__ h,
                                             int64_t h_ms, double2* __restrict__ partial,
                                             int nblk, int64_t n, const int* __restrict__ act) {
    using C = typename CT<T>::t;
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    if (win) win += mem * win_ms;
    if (wd) wd += mem * wd_ms;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __shared__ double2 hs[MAXM + 16];
    __shared__ double2 red[4][CGS_MAXG * 16];
    if (MODE != CGS_DOT) {
        for (int t = threadIdx.x; t < ncols; t += blockDim.x) hs[t] = h[mem * h_ms + t];
        __syncthreads();
    }
    const int nval = MODE == CGS_DOT ? ncols + 1 : (MODE == CGS_UPDATE_DOT ? ncols : 1);
    const int ngrp = (nval + 15) / 16;
    double2 acc[CGS_MAXG];
#pragma unroll
    for (int g = 0; g < CGS_MAXG; ++g) acc[g] = mk(0, 0);
    double nacc = 0;

    const int64_t ntiles = (n + 63) / 64;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t i = tile * 64 + lane;
        const bool ok = i < n;
        if (MODE == CGS_DOT) {
            double2 w = ok ? to_d(win[i]) : mk(0, 0);
            const double ww = cabs2(w);
#pragma unroll
            for (int g = 0; g < CGS_MAXG; ++g) {
                if (g < ngrp) {
                    double2 a[16];
#pragma unroll
                    for (int c = 0; c < 16; ++c) {
                        const int col = g * 16 + c;
                        if (col < ncols && ok)
                            a[c] = cjmul(to_d(V[col * ldv + i]), w);
                        else
                            a[c] = mk(col == ncols ? ww : 0.0, 0);
                    }
                    acc[g] = cadd(acc[g], rs16(a, lane));
                }
            }
        } else {
            double2 w;
            if (MODE == CGS_UPDATE_DOT || (MODE == CGS_UPDATE && win))
                w = ok ? to_d(win[i]) : mk(0, 0);
            else
                w = ok ? wd[i] : mk(0, 0);
            C vr[CACHE ? MAXM : 1];
            if (CACHE) {
#pragma unroll
                for (int col = 0; col < MAXM; ++col) {
                    if (col < ncols) {
                        vr[col] = ok ? V[col * ldv + i] : C{0, 0};
                        w = csub(w, cmul(to_d(vr[col]), hs[col]));
                    }
                }
            } else {
                for (int col = 0; col < ncols; ++col) {
                    double2 vv = ok ? to_d(V[col * ldv + i]) : mk(0, 0);
                    w = csub(w, cmul(vv, hs[col]));
                }
            }
            if (ok) wd[i] = w;
            if (MODE == CGS_UPDATE_NORM) nacc += cabs2(w);
            if (MODE == CGS_UPDATE_DOT) {
#pragma unroll
                for (int g = 0; g < CGS_MAXG; ++g) {
                    if (g < ngrp) {
                        double2 a[16];
#pragma unroll
                        for (int c = 0; c < 16; ++c) {
                            const int col = g * 16 + c;
                            if (col < ncols && ok) {
                                double2 vv;
                                if (CACHE) vv = to_d(vr[col < MAXM ? col : 0]);
                                else vv = to_d(V[col * ldv + i]);
                                a[c] = cjmul(vv, w);
                            } else {
                                a[c] = mk(0, 0);
                            }
                        }
                        acc[g] = cadd(acc[g], rs16(a, lane));
                    }
                }
            }
        }
    }
    if (MODE == CGS_UPDATE) return;
    // block reduction in a fixed order
    if (MODE == CGS_UPDATE_NORM) {
        nacc = wsum(nacc);
        if (lane == 0) red[wv][0] = mk(nacc, 0);
    } else {
        if ((lane & 3) == 0) {
#pragma unroll
            for (int g = 0; g < CGS_MAXG; ++g)
                if (g < ngrp) red[wv][g * 16 + (lane >> 2)] = acc[g];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nval; t += blockDim.x) {
        double2 s = red[0][t];
        s = cadd(s, red[1][t]);
        s = cadd(s, red[2][t]);
        s = cadd(s, red[3][t]);
        partial[((int64_t)mem * nval + t) * nblk + blockIdx.x] = s;
    }
}

// Orders this wavefront's LDS writes before its own later LDS reads (the
// lanes of one wavefront exchange data through LDS without a block barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP32 basis, passes that need V^H w (DOT and UPDATE_DOT). Each wavefront
// owns 64-row tiles: with lanes = rows it loads the tile's basis entries
// (one coalesced 512 B segment per column, all columns issued before use,
// the next tile's loads issued before the current tile's dot products),
// applies the update w -= V h, and stages the tile in LDS; then with
// lanes = columns each lane accumulates its column's dot product over the
// tile's 64 rows, so no cross-lane reduction is needed until the end.
constexpr int TPAD = MAXM + 1;   // LDS tile row stride (odd: conflict-free both ways)
constexpr int TW_WAVES = 4;

template <typename TW, int MODE>
__global__ __launch_bounds__(64 * TW_WAVES) void k_cgs_tile(
    const float2* __restrict__ V, int64_t ldv, int64_t v_ms, int ncols,
    const typename CT<TW>::t* __restrict__ win, int64_t win_ms, double2* __restrict__ wd,
    int64_t wd_ms, const double2* __restrict__ h, int64_t h_ms, double2* __restrict__ partial,
    int nblk, int64_t n, const int* __restrict__ act) {
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    win += mem * win_ms;
    if (wd) wd += mem * wd_ms;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __shared__ double2 hs[MAXM];
    __shared__ float2 tile[TW_WAVES][64 * TPAD];
    __shared__ double2 wp[TW_WAVES][64];
    __shared__ double2 red[TW_WAVES][MAXM + 1];
    if (MODE == CGS_UPDATE_DOT)
        for (int t = threadIdx.x; t < MAXM; t += blockDim.x)
            hs[t] = t < ncols ? h[mem * h_ms + t] : mk(0, 0);
    __syncthreads();
    float2* tl = tile[wv];
    double2 acc = mk(0, 0);
    double nacc = 0;
    const int64_t ntiles = (n + 63) / 64;
    const int64_t stride = (int64_t)gridDim.x * TW_WAVES;
    int64_t t = (int64_t)blockIdx.x * TW_WAVES + wv;
    // Basis allocations carry 8 spare columns, so the loads run in uniform
    // chunks of 8 columns; rows past n are clamped to a valid row and enter
    // with weight zero.
    float2 vr[MAXM];
    typename CT<TW>::t wn;
    auto load_tile = [&](int64_t tt) {
        int64_t i = tt * 64 + lane;
        if (i >= n) i = n - 1;
        wn = win[i];
        const float2* p = V + i;
#pragma unroll
        for (int c8 = 0; c8 < MAXM; c8 += 8) {
            if (c8 < ncols) {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    vr[c8 + c] = *p;
                    p += ldv;
                }
            }
        }
    };
    if (t < ntiles) load_tile(t);
    for (; t < ntiles; t += stride) {
        const int64_t i = t * 64 + lane;
        const bool ok = i < n;
        double2 w = ok ? to_d(wn) : mk(0, 0);
        if (MODE == CGS_DOT) nacc += cabs2(w);
#pragma unroll
        for (int c8 = 0; c8 < MAXM; c8 += 8) {
            if (c8 < ncols) {
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    if (MODE == CGS_UPDATE_DOT) w = csub(w, cmul(to_d(vr[c8 + c]), hs[c8 + c]));
                    tl[lane * TPAD + c8 + c] = vr[c8 + c];
                }
            }
        }
        if (MODE == CGS_UPDATE_DOT && ok) wd[i] = w;
        wp[wv][lane] = ok ? w : mk(0, 0);
        // prefetch the next tile while this one's dot products run
        if (t + stride < ntiles) load_tile(t + stride);
        wave_sync();
        if (lane < ncols) {
#pragma unroll 8
            for (int r = 0; r < 64; ++r) acc = cadd(acc, cjmul(to_d(tl[r * TPAD + lane]), wp[wv][r]));
        }
        wave_sync();
    }
    if (lane < ncols) red[wv][lane] = acc;
    if (MODE == CGS_DOT) {
        nacc = wsum(nacc);
        if (lane == 0) red[wv][ncols] = mk(nacc, 0);
    }
    __syncthreads();
    const int nval = MODE == CGS_DOT ? ncols + 1 : ncols;
    for (int c = threadIdx.x; c < nval; c += blockDim.x) {
        double2 sum = red[0][c];
        for (int ww = 1; ww < TW_WAVES; ++ww) sum = cadd(sum, red[ww][c]);
        partial[((int64_t)mem * nval + c) * nblk + blockIdx.x] = sum;
    }
}

// Streaming passes without dot products (UPDATE, UPDATE_NORM) for both
// precisions: lanes = rows, all of a row's basis entries loaded before use.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_cgs_stream(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int64_t v_ms, int ncols,
    const typename CT<T>::t* __restrict__ win, int64_t win_ms, double2* __restrict__ wd,
    int64_t wd_ms, const double2* __restrict__ h, int64_t h_ms, double2* __restrict__ partial,
    int nblk, int64_t n, const int* __restrict__ act) {
    using C = typename CT<T>::t;
    constexpr int CH = std::is_same<T, float>::value ? 32 : 16;
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    if (win) win += mem * win_ms;
    wd += mem * wd_ms;
    __shared__ double2 hs[MAXM];
    __shared__ double red[4];
    for (int t = threadIdx.x; t < ncols; t += blockDim.x) hs[t] = h[mem * h_ms + t];
    __syncthreads();
    double nacc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 w = win ? to_d(win[i]) : wd[i];
        for (int c0 = 0; c0 < ncols; c0 += CH) {
            C vr[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (c0 + c < ncols) vr[c] = V[(c0 + c) * ldv + i];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (c0 + c < ncols) w = csub(w, cmul(to_d(vr[c]), hs[c0 + c]));
        }
        wd[i] = w;
        if (MODE == CGS_UPDATE_NORM) nacc += cabs2(w);
    }
    if (MODE != CGS_UPDATE_NORM) return;
    nacc = wsum(nacc);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = nacc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(int64_t)mem * nblk + blockIdx.x] = mk(red[0] + red[1] + red[2] + red[3], 0);
}

template <typename T, typename TW>
void cgs_pass(int mode, const typename CT<T>::t* V, int64_t ldv, int64_t v_mstride, int ncols,
              const typename CT<TW>::t* win, int64_t win_mstride, double2* wd, int64_t wd_mstride,
              const double2* h, int64_t h_mstride, double2* partial, int nblk, int64_t n, int nmem,
              hipStream_t st, const int* act) {
    dim3 grid(nblk, nmem), blk(CGS_BLOCK);
    if (mode == CGS_UPDATE_NORM || mode == CGS_UPDATE) {
        // streaming passes read win only as type T (never the FP64 residual)
        const typename CT<T>::t* wt = (const typename CT<T>::t*)win;
        if (mode == CGS_UPDATE_NORM)
            hipLaunchKernelGGL((k_cgs_stream<T, CGS_UPDATE_NORM>), grid, blk, 0, st, V, ldv,
                               v_mstride, ncols, wt, win_mstride, wd, wd_mstride, h, h_mstride,
                               partial, nblk, n, act);
        else
            hipLaunchKernelGGL((k_cgs_stream<T, CGS_UPDATE>), grid, blk, 0, st, V, ldv, v_mstride,
                               ncols, wt, win_mstride, wd, wd_mstride, h, h_mstride, partial, nblk,
                               n, act);
        return;
    }
    if constexpr (std::is_same<T, float>::value) {
        dim3 bt(64 * TW_WAVES);
        if (mode == CGS_DOT)
            hipLaunchKernelGGL((k_cgs_tile<TW, CGS_DOT>), grid, bt, 0, st, V, ldv, v_mstride,
                               ncols, win, win_mstride, wd, wd_mstride, h, h_mstride, partial,
                               nblk, n, act);
        else
            hipLaunchKernelGGL((k_cgs_tile<TW, CGS_UPDATE_DOT>), grid, bt, 0, st, V, ldv,
                               v_mstride, ncols, win, win_mstride, wd, wd_mstride, h, h_mstride,
                               partial, nblk, n, act);
    } else {
#define GDR_CGS(M)                                                                               \
    hipLaunchKernelGGL((k_cgs<T, TW, M, false>), grid, blk, 0, st, V, ldv, v_mstride, ncols, win, \
                       win_mstride, wd, wd_mstride, h, h_mstride, partial, nblk, n, act)
        if (mode == CGS_DOT) GDR_CGS(CGS_DOT);
        else GDR_CGS(CGS_UPDATE_DOT);
#undef GDR_CGS
    }
}
template void cgs_pass<double, double>(int, const double2*, int64_t, int64_t, int, const double2*,
                                       int64_t, double2*, int64_t, const double2*, int64_t,
                                       double2*, int, int64_t, int, hipStream_t, const int*);
template void cgs_pass<float, float>(int, const float2*, int64_t, int64_t, int, const float2*,
                                     int64_t, double2*, int64_t, const double2*, int64_t, double2*,
                                     int, int64_t, int, hipStream_t, const int*);
template void cgs_pass<float, double>(int, const float2*, int64_t, int64_t, int, const double2*,
                                      int64_t, double2*, int64_t, const double2*, int64_t, double2*,
                                      int, int64_t, int, hipStream_t, const int*);

// ---------------------------------------------------------------------------
// Delayed classical Gram-Schmidt (DCGS2) passes of the Arnoldi step.
//
// k_gs_dot: one sweep over V forms V_{0..nc-1}^H x_a for NX right-hand
// vectors x_a, plus ||x_{NX-1}||^2. A block owns a contiguous row range; its
// four waves split the columns, each wave accumulates up to 8 columns x NX
// vectors per lane in FP64 over the rows, then a butterfly reduce-scatter
// over the wavefront leaves one sum per four lanes. Partial sums go to
// partial[((mem*nval) + a*nc + c)*nblk + blk], nval = NX*nc + 1.
template <typename T, typename TX, int NX>
__global__ __launch_bounds__(256) void k_gs_dot(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int64_t v_ms, int nc,
    const typename CT<TX>::t* __restrict__ x0, int64_t x0_ms,
    const typename CT<TX>::t* __restrict__ x1, int64_t x1_ms, double2* __restrict__ partial,
    int nblk, int64_t n, const int* __restrict__ act) {
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    x0 += mem * x0_ms;
    if (NX > 1) x1 += mem * x1_ms;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int64_t per = ((n + nblk - 1) / nblk + 63) & ~(int64_t)63;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    const int nval = NX * nc + 1;
    double2* pout = partial + (int64_t)mem * nval * nblk + blockIdx.x;
    const int g = (nc + 3) >> 2;
    const int c0 = wv * g;
    const int c1 = c0 + g < nc ? c0 + g : nc;
    for (int cs = c0; cs < c1; cs += 8) {
        const int cnt = c1 - cs < 8 ? c1 - cs : 8;
        double2 acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = mk(0, 0);
        const typename CT<T>::t* vp = V + (int64_t)cs * ldv;
        for (int64_t i = r0 + lane; i < r1; i += 64) {
            const double2 xa = to_d(x0[i]);
            const double2 xb = NX > 1 ? to_d(x1[i]) : mk(0, 0);
            typename CT<T>::t vr[8];
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < cnt) vr[c] = vp[(int64_t)c * ldv + i];
#pragma unroll
            for (int c = 0; c < 8; ++c)
                if (c < cnt) {
                    const double2 v = to_d(vr[c]);
                    acc[c] = cadd(acc[c], cjmul(v, xa));
                    if (NX > 1) acc[8 + c] = cadd(acc[8 + c], cjmul(v, xb));
                }
        }
        const double2 sum = rs16(acc, lane);
        if ((lane & 3) == 0) {
            const int q = (lane >> 2) & 15;
            const int a = q >> 3, c = q & 7;
            if (c < cnt && a < NX) pout[(int64_t)(a * nc + cs + c) * nblk] = sum;
        }
    }
    if (wv == 3) {
        const typename CT<TX>::t* xl = NX > 1 ? x1 : x0;
        double s2 = 0;
        for (int64_t i = r0 + lane; i < r1; i += 64) s2 += cabs2(to_d(xl[i]));
        s2 = wsum(s2);
        if (lane == 0) pout[(int64_t)(NX * nc) * nblk] = mk(s2, 0);
    }
}

// k_gs_update: one sweep forms NO outputs
//   y_o = sum_a beta[o][a] x_a - sum_{c<nc} V_c coef[o][c]
// with coefficients coef[mem*coef_ms + o*(MAXM+1) + c] and
// beta[mem*coef_ms + 2*(MAXM+1) + 2*o + a]. y_0 may alias x_0 (each row is
// read before it is written by the same thread).
template <typename T, int NX, int NO>
__global__ __launch_bounds__(256) void k_gs_update(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int64_t v_ms, int nc,
    const typename CT<T>::t* x0, int64_t x0_ms, const typename CT<T>::t* __restrict__ x1,
    int64_t x1_ms, typename CT<T>::t* y0, int64_t y0_ms, typename CT<T>::t* __restrict__ y1,
    int64_t y1_ms, const double2* __restrict__ coef, int64_t coef_ms, int64_t n,
    const int* __restrict__ act) {
    using C = typename CT<T>::t;
    constexpr int CH = std::is_same<T, float>::value ? 16 : 8;
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    x0 += mem * x0_ms;
    y0 += mem * y0_ms;
    if (NX > 1) x1 += mem * x1_ms;
    if (NO > 1) y1 += mem * y1_ms;
    coef += mem * coef_ms;
    __shared__ double2 cf[NO][MAXM + 1];
    __shared__ double2 bt[NO][2];
    for (int t = threadIdx.x; t < nc; t += blockDim.x) {
        cf[0][t] = coef[t];
        if (NO > 1) cf[NO - 1][t] = coef[(MAXM + 1) + t];
    }
    if (threadIdx.x < 2 * NO) bt[threadIdx.x >> 1][threadIdx.x & 1] = coef[2 * (MAXM + 1) + threadIdx.x];
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 xa = to_d(x0[i]);
        const double2 xb = NX > 1 ? to_d(x1[i]) : mk(0, 0);
        double2 o0 = cmul(bt[0][0], xa), o1 = mk(0, 0);
        if (NX > 1) o0 = cadd(o0, cmul(bt[0][1], xb));
        if (NO > 1) o1 = cadd(cmul(bt[NO - 1][0], xa), cmul(bt[NO - 1][1], xb));
        for (int cb = 0; cb < nc; cb += CH) {
            C vr[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (cb + c < nc) vr[c] = V[(int64_t)(cb + c) * ldv + i];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (cb + c < nc) {
                    const double2 v = to_d(vr[c]);
                    o0 = csub(o0, cmul(v, cf[0][cb + c]));
                    if (NO > 1) o1 = csub(o1, cmul(v, cf[NO - 1][cb + c]));
                }
        }
        y0[i] = from_d<T>(o0);
        if (NO > 1) y1[i] = from_d<T>(o1);
    }
}

template <typename T, typename TX>
void gs_dot(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
            const typename CT<TX>::t* x0, int64_t x0_ms, const typename CT<TX>::t* x1,
            int64_t x1_ms, double2* partial, int nblk, int64_t n, int nmem, hipStream_t st,
            const int* act) {
    dim3 grid(nblk, nmem), blk(256);
    if (x1)
        hipLaunchKernelGGL((k_gs_dot<T, TX, 2>), grid, blk, 0, st, V, ldv, v_ms, nc, x0, x0_ms, x1,
                           x1_ms, partial, nblk, n, act);
    else
        hipLaunchKernelGGL((k_gs_dot<T, TX, 1>), grid, blk, 0, st, V, ldv, v_ms, nc, x0, x0_ms, x1,
                           x1_ms, partial, nblk, n, act);
}

template <typename T>
void gs_update(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
               const typename CT<T>::t* x0, int64_t x0_ms, const typename CT<T>::t* x1,
               int64_t x1_ms, typename CT<T>::t* y0, int64_t y0_ms, typename CT<T>::t* y1,
               int64_t y1_ms, const double2* coef, int64_t coef_ms, int64_t n, int nmem,
               hipStream_t st, const int* act) {
    dim3 grid(cgs_nblk(n), nmem), blk(256);
    if (x1)
        hipLaunchKernelGGL((k_gs_update<T, 2, 2>), grid, blk, 0, st, V, ldv, v_ms, nc, x0, x0_ms,
                           x1, x1_ms, y0, y0_ms, y1, y1_ms, coef, coef_ms, n, act);
    else
        hipLaunchKernelGGL((k_gs_update<T, 1, 1>), grid, blk, 0, st, V, ldv, v_ms, nc, x0, x0_ms,
                           x1, x1_ms, y0, y0_ms, y1, y1_ms, coef, coef_ms, n, act);
}

template void gs_dot<float, float>(const float2*, int64_t, int64_t, int, const float2*, int64_t,
                                   const float2*, int64_t, double2*, int, int64_t, int,
                                   hipStream_t, const int*);
template void gs_dot<double, double>(const double2*, int64_t, int64_t, int, const double2*,
                                     int64_t, const double2*, int64_t, double2*, int, int64_t,
                                     int, hipStream_t, const int*);
template void gs_dot<float, double>(const float2*, int64_t, int64_t, int, const double2*, int64_t,
                                    const double2*, int64_t, double2*, int, int64_t, int,
                                    hipStream_t, const int*);
template void gs_update<float>(const float2*, int64_t, int64_t, int, const float2*, int64_t,
                               const float2*, int64_t, float2*, int64_t, float2*, int64_t,
                               const double2*, int64_t, int64_t, int, hipStream_t, const int*);
template void gs_update<double>(const double2*, int64_t, int64_t, int, const double2*, int64_t,
                                const double2*, int64_t, double2*, int64_t, double2*, int64_t,
                                const double2*, int64_t, int64_t, int, hipStream_t, const int*);

// DCGS2 bookkeeping for step j (one wavefront per member). G holds the reduced
// sums of k_gs_dot over columns 0..j with x_0 = r (the once-orthogonalised,
// unnormalised candidate in column j) and, when nx = 2, x_1 = w = A r:
//   s = V_j^H r, alpha = r^H r, p = V_j^H w, gamma = r^H w, omega = ||w||^2.
// With nu = (alpha - ||s||^2)^{1/2} the candidate becomes q_j = (r - V_j s)/nu,
// column j-1 of H gains its second Gram-Schmidt pass (H[0..j-1][j-1] += s,
// H[j][j-1] = nu) unless `first`, and for nx = 2 the first pass of the next
// column follows from the same sums: with d = [p; (gamma - s^H p)/nu],
//   H[0..j][j] = (d - H[0..j][0..j-1] s)/nu,
//   r_next = (w - V_j p - d_j q_j)/nu.
// Output coefficients for k_gs_update (q_j and r_next as combinations of r, w
// and V_j). A subdiagonal nu <= tol * ||A q_{j-1}|| is a breakdown at column j-1:
// brk is set and every coefficient of this and later steps is zero.
__global__ __launch_bounds__(64) void k_dcgs_coef(const double2* __restrict__ G, int64_t g_ms,
                                                  int j, int nx, int first, double2* __restrict__ H,
                                                  int64_t ldh, int64_t h_ms,
                                                  double2* __restrict__ coef, int64_t coef_ms,
                                                  double* __restrict__ ref, int* __restrict__ brk,
                                                  double tol, const int* __restrict__ act) {
    const int b = blockIdx.x;
    if (act && !act[b]) return;
    const int lane = threadIdx.x;
    G += b * g_ms;
    H += b * h_ms;
    coef += b * coef_ms;
    const int nc = j + 1;
    __shared__ double2 ss[MAXM + 1];
    const double2 s = lane < j ? G[lane] : mk(0, 0);
    const double2 pk = (nx > 1 && lane < j) ? G[nc + lane] : mk(0, 0);
    ss[lane] = s;
    const double alpha = G[j].x;
    const double nrm_s = wsum(cabs2(s));
    const double nu2 = alpha - nrm_s;
    const double refv = first ? 0.0 : ref[b];
    bool broken = brk[b] >= 0;
    if (!broken && !(nu2 > tol * tol * refv * refv && nu2 > 0)) {
        broken = true;
        if (lane == 0) brk[b] = j - 1;
        if (!first && lane == 0) H[(int64_t)(j - 1) * ldh + j] = mk(0, 0);
    }
    if (broken) {
        for (int t = lane; t < 2 * (MAXM + 1) + 4; t += 64) coef[t] = mk(0, 0);
        if (nx > 1)
            for (int i = lane; i <= j; i += 64) H[(int64_t)j * ldh + i] = mk(0, 0);
        if (lane == 0) ref[b] = 0;
        return;
    }
    const double nu = sqrt(nu2), inu = 1.0 / nu;
    if (!first) {
        if (lane < j) {
            double2* hc = H + (int64_t)(j - 1) * ldh;
            hc[lane] = cadd(hc[lane], s);
        }
        if (lane == 0) H[(int64_t)(j - 1) * ldh + j] = mk(nu, 0);
    }
    if (lane < j) coef[lane] = cscale(s, inu);
    if (lane == 0) {
        coef[2 * (MAXM + 1) + 0] = mk(inu, 0);
        coef[2 * (MAXM + 1) + 1] = mk(0, 0);
    }
    if (nx == 1) return;
    __syncthreads();   // corrected column j-1 visible to every lane
    const double2 sp = mk(wsum(s.x * pk.x + s.y * pk.y), wsum(s.x * pk.y - s.y * pk.x));
    const double2 gam = G[nc + j];
    const double2 dj = cscale(csub(gam, sp), inu);
    // H[0..j][j] = (d - H s)/nu, lane i = row i
    for (int i = lane; i <= j; i += 64) {
        double2 hs = mk(0, 0);
        // full sum: after a GMRES-DR restart the leading (k+1) x k block is dense
        for (int kk = 0; kk < j; ++kk) hs = cadd(hs, cmul(H[(int64_t)kk * ldh + i], ss[kk]));
        const double2 di = i < j ? G[nc + i] : dj;
        H[(int64_t)j * ldh + i] = cscale(csub(di, hs), inu);
    }
    const double2 djn = cscale(dj, inu);
    if (lane < j) coef[(MAXM + 1) + lane] = cscale(csub(pk, cmul(djn, s)), inu);
    if (lane == 0) {
        coef[2 * (MAXM + 1) + 2] = cscale(djn, -inu);
        coef[2 * (MAXM + 1) + 3] = mk(inu, 0);
        ref[b] = sqrt(G[2 * nc].x) * inu;
    }
}

void dcgs_coef(const double2* G, int64_t g_ms, int j, int nx, int first, double2* H, int64_t ldh,
               int64_t h_ms, double2* coef, int64_t coef_ms, double* ref, int* brk, double tol,
               int nmem, hipStream_t st, const int* act) {
    hipLaunchKernelGGL(k_dcgs_coef, dim3(nmem), dim3(64), 0, st, G, g_ms, j, nx, first, H, ldh,
                       h_ms, coef, coef_ms, ref, brk, tol, act);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_cols(const double2* __restrict__ partial, int nblk,
                                                     int ncols, double2* __restrict__ out,
                                                     int64_t out_ms, double2* __restrict__ add_to,
                                                     int64_t add_ms, const int* __restrict__ act) {
    const int c = blockIdx.x, b = blockIdx.y;
    if (act && !act[b]) return;
    const double2* p = partial + ((int64_t)b * ncols + c) * nblk;
    double2 s = mk(0, 0);
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) s = cadd(s, p[k]);
    __shared__ double2 red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (out) out[b * out_ms + c] = red[0];
        if (add_to) add_to[b * add_ms + c] = cadd(add_to[b * add_ms + c], red[0]);
    }
}

void reduce_cols(const double2* partial, int nblk, int ncols, double2* out, int64_t out_mstride,
                 double2* add_to, int64_t add_mstride, int nmem, hipStream_t st,
                 const int* act) {
    hipLaunchKernelGGL(k_reduce_cols, dim3(ncols, nmem), dim3(256), 0, st, partial, nblk, ncols,
                       out, out_mstride, add_to, add_mstride, act);
}

__global__ __launch_bounds__(256) void k_norm_finish(const double2* __restrict__ partial, int nblk,
                                                     double2* __restrict__ H, int64_t ldh,
                                                     int64_t h_ms, int j,
                                                     const double2* __restrict__ w0, int64_t w0_ms,
                                                     double* __restrict__ inv, int* __restrict__ brk,
                                                     double tol_rel, const int* __restrict__ act) {
    const int b = blockIdx.x;
    if (act && !act[b]) return;
    const double2* p = partial + (int64_t)b * nblk;
    double s = 0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) s += p[k].x;
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double nrm = sqrt(red[0]);
        double ref = sqrt(w0[b * w0_ms].x);
        bool broke = brk[b] >= 0 || !(nrm > tol_rel * ref);
        if (broke) {
            if (brk[b] < 0) brk[b] = j;
            H[b * h_ms + (int64_t)j * ldh + j + 1] = mk(0, 0);
            inv[b] = 0.0;
        } else {
            H[b * h_ms + (int64_t)j * ldh + j + 1] = mk(nrm, 0);
            inv[b] = 1.0 / nrm;
        }
    }
}

void norm_finish(const double2* partial, int nblk, double2* H, int64_t ldh, int64_t h_mstride,
                 int j, const double2* w0, int64_t w0_mstride, double* inv, int* brk,
                 double tol_rel, int nmem, hipStream_t st, const int* act) {
    hipLaunchKernelGGL(k_norm_finish, dim3(nmem), dim3(256), 0, st, partial, nblk, H, ldh,
                       h_mstride, j, w0, w0_mstride, inv, brk, tol_rel, act);
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_scale_store(const double2* __restrict__ wd, int64_t wd_ms,
                                                     const double* __restrict__ inv,
                                                     typename CT<T>::t* __restrict__ v,
                                                     int64_t v_ms, int64_t n,
                                                     const int* __restrict__ act) {
    const int b = blockIdx.y;
    if (act && !act[b]) return;
    const double s = inv[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        v[b * v_ms + i] = from_d<T>(cscale(wd[b * wd_ms + i], s));
}

static int vec_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g > 8192 ? 8192 : g);
}

template <typename T>
void scale_store(const double2* wd, int64_t wd_mstride, const double* inv,
                 typename CT<T>::t* v, int64_t v_mstride, int64_t n, int nmem, hipStream_t st,
                 const int* act) {
    hipLaunchKernelGGL(k_scale_store<T>, dim3(vec_grid(n), nmem), dim3(256), 0, st, wd,
                       wd_mstride, inv, v, v_mstride, n, act);
}
template void scale_store<double>(const double2*, int64_t, const double*, double2*, int64_t,
                                  int64_t, int, hipStream_t, const int*);
template void scale_store<float>(const double2*, int64_t, const double*, float2*, int64_t, int64_t,
                                 int, hipStream_t, const int*);

template <typename T>
__global__ __launch_bounds__(256) void k_convert_scale(const double2* __restrict__ x, int64_t x_ms,
                                                       const double* __restrict__ scal, int sc_stride,
                                                       typename CT<T>::t* __restrict__ y,
                                                       int64_t y_ms, int64_t n,
                                                       const int* __restrict__ act) {
    const int b = blockIdx.y;
    if (act && !act[b]) return;
    const double s = scal ? scal[b * sc_stride] : 1.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[b * y_ms + i] = from_d<T>(cscale(x[b * x_ms + i], s));
}

template <typename T>
void convert_scale(const double2* x, int64_t x_mstride, const double* scal, int sc_stride,
                   typename CT<T>::t* y, int64_t y_mstride, int64_t n, int nmem, hipStream_t st,
                   const int* act) {
    hipLaunchKernelGGL(k_convert_scale<T>, dim3(vec_grid(n), nmem), dim3(256), 0, st, x,
                       x_mstride, scal, sc_stride, y, y_mstride, n, act);
}
template void convert_scale<double>(const double2*, int64_t, const double*, int, double2*, int64_t,
                                    int64_t, int, hipStream_t, const int*);
template void convert_scale<float>(const double2*, int64_t, const double*, int, float2*, int64_t,
                                   int64_t, int, hipStream_t, const int*);

__global__ __launch_bounds__(256) void k_axpy_dev(double2* __restrict__ x, int64_t x_ms,
                                                  const double2* __restrict__ y, int64_t y_ms,
                                                  const double2* __restrict__ coef, int cstride,
                                                  int64_t n, const int* __restrict__ act) {
    const int b = blockIdx.y;
    if (act && !act[b]) return;
    const double2 a = coef ? coef[b * cstride] : mk(1, 0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[b * x_ms + i] = cadd(x[b * x_ms + i], cmul(a, y[b * y_ms + i]));
}
void axpy_dev(double2* x, int64_t x_mstride, const double2* y, int64_t y_mstride,
              const double2* coef, int cstride, int64_t n, int nmem, hipStream_t st,
              const int* act) {
    hipLaunchKernelGGL(k_axpy_dev, dim3(vec_grid(n), nmem), dim3(256), 0, st, x, x_mstride, y,
                       y_mstride, coef, cstride, n, act);
}

__global__ __launch_bounds__(256) void k_scal_dev(double2* __restrict__ x, int64_t x_ms,
                                                  const double2* __restrict__ coef, int64_t n) {
    const int b = blockIdx.y;
    const double2 a = coef[b];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        x[b * x_ms + i] = cmul(a, x[b * x_ms + i]);
}
void scal_dev(double2* x, int64_t x_mstride, const double2* coef, int64_t n, int nmem,
              hipStream_t st) {
    hipLaunchKernelGGL(k_scal_dev, dim3(vec_grid(n), nmem), dim3(256), 0, st, x, x_mstride, coef,
                       n);
}

__global__ __launch_bounds__(256) void k_copy_vec(const double2* __restrict__ x, int64_t x_ms,
                                                  double2* __restrict__ y, int64_t y_ms, int64_t n) {
    const int b = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[b * y_ms + i] = x[b * x_ms + i];
}
void copy_vec(const double2* x, int64_t x_mstride, double2* y, int64_t y_mstride, int64_t n,
              int nmem, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_vec, dim3(vec_grid(n), nmem), dim3(256), 0, st, x, x_mstride, y,
                       y_mstride, n);
}

__global__ void k_start_cycle(const double2* __restrict__ rn2, int64_t rs, double2* __restrict__ c,
                              int64_t cs, int m, double* __restrict__ inv,
                              const int* __restrict__ act) {
    const int b = blockIdx.x;
    if (act && !act[b]) return;
    const double nr = sqrt(rn2[b * rs].x);
    for (int i = threadIdx.x; i <= m; i += blockDim.x) c[b * cs + i] = mk(i == 0 ? nr : 0.0, 0);
    if (threadIdx.x == 0) inv[b] = nr > 0 ? 1.0 / nr : 0.0;
}
void start_cycle(const double2* rn2, int64_t rs, double2* c, int64_t cs, int m, double* inv,
                 int nmem, hipStream_t st, const int* act) {
    hipLaunchKernelGGL(k_start_cycle, dim3(nmem), dim3(64), 0, st, rn2, rs, c, cs, m, inv, act);
}

__global__ void k_fill_int(int* p, int v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
void fill_int(int* p, int v, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, st, p, v, n);
}

// ---------------------------------------------------------------------------
// out_s = keep_s * out_s + sum_l V_l coef[l + s*ldc]
constexpr int VC_MAXOUT = MAXNS + 2;

template <typename T>
__global__ __launch_bounds__(256) void k_vcombine(const typename CT<T>::t* __restrict__ V,
                                                  int64_t ldv, int64_t v_ms, int ncols,
                                                  const double2* __restrict__ coef, int ldc,
                                                  int64_t c_ms, int nout, double2* __restrict__ out,
                                                  int64_t o_stride, int64_t o_ms, unsigned keep,
                                                  int64_t n, const int* __restrict__ act) {
    const int b = blockIdx.y;
    if (act && !act[b]) return;
    V += b * v_ms;
    coef += b * c_ms;
    out += b * o_ms;
    __shared__ double2 cs[(MAXM + 1) * VC_MAXOUT];
    for (int t = threadIdx.x; t < ncols * nout; t += blockDim.x) {
        int l = t % ncols, s = t / ncols;
        cs[t] = coef[l + s * ldc];
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 acc[VC_MAXOUT];
#pragma unroll
        for (int s = 0; s < VC_MAXOUT; ++s) acc[s] = mk(0, 0);
        for (int l = 0; l < ncols; ++l) {
            double2 v = to_d(V[l * ldv + i]);
#pragma unroll
            for (int s = 0; s < VC_MAXOUT; ++s)
                if (s < nout) acc[s] = cadd(acc[s], cmul(v, cs[l + s * ncols]));
        }
#pragma unroll
        for (int s = 0; s < VC_MAXOUT; ++s)
            if (s < nout) {
                double2* o = out + s * o_stride + i;
                *o = ((keep >> s) & 1u) ? cadd(*o, acc[s]) : acc[s];
            }
    }
}

template <typename T>
void vcombine(const typename CT<T>::t* V, int64_t ldv, int64_t v_mstride, int ncols,
              const double2* coef, int ldc, int64_t c_mstride, int nout, double2* out,
              int64_t o_stride, int64_t o_mstride, unsigned keep_mask, int64_t n, int nmem,
              hipStream_t st, const int* act) {
    hipLaunchKernelGGL(k_vcombine<T>, dim3(vec_grid(n), nmem), dim3(256), 0, st, V, ldv,
                       v_mstride, ncols, coef, ldc, c_mstride, nout, out, o_stride, o_mstride,
                       keep_mask, n, act);
}
template void vcombine<double>(const double2*, int64_t, int64_t, int, const double2*, int, int64_t,
                               int, double2*, int64_t, int64_t, unsigned, int64_t, int,
                               hipStream_t, const int*);
template void vcombine<float>(const float2*, int64_t, int64_t, int, const double2*, int, int64_t,
                              int, double2*, int64_t, int64_t, unsigned, int64_t, int, hipStream_t,
                              const int*);

// W_j = sum_l V_l P[l + j*ldp], computed in the storage precision, output
// columns in chunks held in registers.
template <typename T, int CH>
__global__ __launch_bounds__(256) void k_vrecombine(const typename CT<T>::t* __restrict__ V,
                                                    int64_t ldv, int ncols,
                                                    const double2* __restrict__ P, int ldp, int nout,
                                                    typename CT<T>::t* __restrict__ W, int64_t ldw,
                                                    int64_t n) {
    using C = typename CT<T>::t;
    __shared__ C ps[(MAXM + 1) * (MAXM + 1)];
    for (int t = threadIdx.x; t < ncols * nout; t += blockDim.x) {
        int l = t % ncols, j = t / ncols;
        double2 pv = P[l + j * ldp];
        ps[t] = C{(T)pv.x, (T)pv.y};
    }
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int j0 = 0; j0 < nout; j0 += CH) {
            C acc[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) acc[c] = C{0, 0};
            for (int l = 0; l < ncols; ++l) {
                C v = V[l * ldv + i];
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    if (j0 + c < nout) {
                        C pv = ps[l + (j0 + c) * ncols];
                        acc[c].x += v.x * pv.x - v.y * pv.y;
                        acc[c].y += v.x * pv.y + v.y * pv.x;
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (j0 + c < nout) W[(j0 + c) * ldw + i] = acc[c];
        }
    }
}

template <typename T>
void vrecombine(const typename CT<T>::t* V, int64_t ldv, int ncols, const double2* P, int ldp,
                int nout, typename CT<T>::t* W, int64_t ldw, int64_t n, hipStream_t st) {
    constexpr int CH = std::is_same<T, float>::value ? 32 : 16;
    hipLaunchKernelGGL((k_vrecombine<T, CH>), dim3(vec_grid(n)), dim3(256), 0, st, V, ldv, ncols,
                       P, ldp, nout, W, ldw, n);
}
template void vrecombine<double>(const double2*, int64_t, int, const double2*, int, int, double2*,
                                 int64_t, int64_t, hipStream_t);
template void vrecombine<float>(const float2*, int64_t, int, const double2*, int, int, float2*,
                                int64_t, int64_t, hipStream_t);

}  // namespace gdr
