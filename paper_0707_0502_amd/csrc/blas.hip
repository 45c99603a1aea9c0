// Vector kernels of the Arnoldi recurrence (eq. (2.2)): classical Gram-Schmidt
// against the Krylov basis in the delayed two-pass form (DCGS2), norms,
// scaling, and the tall-skinny combinations x_i += V d_i, r = V s and
// V_{k+1} = V_{m+1} P.
//
// Dot products V^H x: lanes own rows, each wave accumulates a group of
// columns over its block's rows in FP64 registers, and a butterfly
// reduce-scatter over the wavefront (shuffles at distance 32,16,8,4, then an
// all-reduce over 2,1) leaves value (lane>>2)&15 on four lanes. Blocks write
// per-column partial sums; a second kernel adds them in a fixed order, so
// every result is bitwise reproducible. All accumulation is FP64.
#include <cstdint>
#include <cstdio>
#include <initializer_list>
#include <stdexcept>
#include <string>

#include "kernels.h"
#include "tune.h"

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

int cgs_nblk(int64_t n, int nmem, bool wide) {
    int64_t tiles = (n + 63) / 64;
    int64_t nb = (tiles + 7) / 8;   // >= 2 tiles per wave on average
    // one FP32 member alone on the chip keeps more loads in flight with 2048
    // blocks; batched members already fill it with 1024 each
    const int64_t cap = wide && nmem == 1 ? 2048 : 1024;
    if (nb > cap) nb = cap;
    if (nb < 1) nb = 1;
    return (int)nb;
}

// Blocks per member of a row sweep whose rows are independent (update sweeps):
// candidate 0 is cgs_nblk's choice, 1..3 other caps on the blocks per member.
constexpr int SWEEP_NCAND = 4;
static int sweep_nblk(int64_t n, int nmem, bool wide, int cand) {
    const int dflt = cgs_nblk(n, nmem, wide);
    if (cand <= 0 || cand >= SWEEP_NCAND) return dflt;
    const int64_t alt = wide && nmem == 1 ? 1024 : 2048;
    const int64_t caps[3] = {512, alt, 4096};
    int64_t nb = ((n + 63) / 64 + 7) / 8;
    if (nb > caps[cand - 1]) nb = caps[cand - 1];
    return (int)(nb < 1 ? 1 : nb);
}

// tuning key of a row sweep: rows, members, vectors per pass, rows per lane
static std::string sweep_shape(int64_t n, int nmem, int nx, bool r2) {
    char b[64];
    std::snprintf(b, sizeof b, "%lld|%d|%d|%d", (long long)n, nmem, nx, r2 ? 2 : 1);
    return b;
}

// ---------------------------------------------------------------------------
// Row access of the sweeps. R = 2 (FP32 data only): a lane owns two adjacent
// complex rows and moves them as one 16-byte access; R = 1: one complex row
// (8 bytes FP32, 16 bytes FP64). The basis V is streamed once per sweep and
// not reused before it would be evicted, so its loads are non-temporal.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

template <typename T, int R> struct RowIO;
template <> struct RowIO<float, 1> {
    using V = float2;
    static __device__ __forceinline__ V ld(const float2* p) { return *p; }
    static __device__ __forceinline__ V ldnt(const float2* p) {
        const f2v v = __builtin_nontemporal_load((const f2v*)p);
        return make_float2(v.x, v.y);
    }
    static __device__ __forceinline__ void get(const V& v, double2* d) { d[0] = to_d(v); }
    static __device__ __forceinline__ void put(float2* p, const double2* d) { *p = from_d<float>(d[0]); }
};
template <> struct RowIO<float, 2> {
    using V = float4;
    static __device__ __forceinline__ V ld(const float2* p) { return *(const float4*)p; }
    static __device__ __forceinline__ V ldnt(const float2* p) {
        const f4v v = __builtin_nontemporal_load((const f4v*)p);
        return make_float4(v.x, v.y, v.z, v.w);
    }
    static __device__ __forceinline__ void get(const V& v, double2* d) {
        d[0] = mk(v.x, v.y);
        d[1] = mk(v.z, v.w);
    }
    static __device__ __forceinline__ void put(float2* p, const double2* d) {
        const float2 a = from_d<float>(d[0]), b = from_d<float>(d[1]);
        *(float4*)p = make_float4(a.x, a.y, b.x, b.y);
    }
};
template <> struct RowIO<double, 1> {
    using V = double2;
    static __device__ __forceinline__ V ld(const double2* p) { return *p; }
    static __device__ __forceinline__ V ldnt(const double2* p) {
        const d2v v = __builtin_nontemporal_load((const d2v*)p);
        return mk(v.x, v.y);
    }
    static __device__ __forceinline__ void get(const V& v, double2* d) { d[0] = v; }
    static __device__ __forceinline__ void put(double2* p, const double2* d) { *p = d[0]; }
};

// 16-byte row pairs need even sizes and strides and 16-byte aligned bases
static inline bool pairable(int64_t n, std::initializer_list<int64_t> strides,
                            std::initializer_list<const void*> ptrs) {
    if (n & 1) return false;
    for (int64_t s : strides)
        if (s & 1) return false;
    for (const void* p : ptrs)
        if (p && ((uintptr_t)p & 15)) return false;
    return true;
}

// Element i of a row array at a uniform base, addressed by a 32-bit byte
// offset (callers keep i * sizeof(P) below 2^32): the global access then
// takes the base in scalar registers and one 32-bit offset per lane, so a run
// of stores needs no 64-bit address registers between them (reusing the
// registers of a store still in flight costs a wait for all memory
// operations of the wave).
template <class P>
static __device__ __forceinline__ P* at32(P* base, int64_t i) {
    return (P*)((char*)base + (uint32_t)((uint64_t)i * sizeof(P)));
}
// a ? x : y on the components (a select of whole array elements can turn
// into an indexed access that moves the array to scratch memory)
static __device__ __forceinline__ double2 csel(bool a, double2 x, double2 y) {
    return mk(a ? x.x : y.x, a ? x.y : y.y);
}
// rows per launch of the kernels that use at32 (2^27 rows of 16 bytes)
constexpr int64_t AT32_ROWS = int64_t(1) << 27;

// ---------------------------------------------------------------------------
// Delayed classical Gram-Schmidt (DCGS2) passes of the Arnoldi step.
//
// k_gs_dot: one sweep over V forms V_{0..nc-1}^H x_a for NX right-hand
// vectors x_a (NX = 2: r_j and w = A r_j) plus ||x_{NX-1}||^2, as per-block
// partial sums (value v of member b at partial[(b*nval + v)*nblk + block],
// nval = NX*nc + 1). A block owns a contiguous row range; its four waves
// split the columns, each wave sweeping its rows for CW columns at a time.
template <typename T, typename TX, int NX, int R>
__global__ __launch_bounds__(256) void k_gs_dot(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int64_t v_ms, int nc,
    const typename CT<TX>::t* __restrict__ x0, int64_t x0_ms,
    const typename CT<TX>::t* __restrict__ x1, int64_t x1_ms, double2* __restrict__ partial,
    int nblk, int64_t n, const int* __restrict__ act) {
    using IV = RowIO<T, R>;
    using IX = RowIO<TX, R>;
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    x0 += mem * x0_ms;
    if (NX > 1) x1 += mem * x1_ms;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int RW = 64 * R;   // rows per wave iteration
    const int64_t per = ((n + nblk - 1) / nblk + RW - 1) / RW * RW;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    const int nval = NX * nc + 1;
    double2* pout = partial + (int64_t)mem * nval * nblk + blockIdx.x;
    // columns per accumulation pass: 2 vectors x 6 columns keep the FP64
    // accumulators within 4 waves per SIMD
    constexpr int CW = NX > 1 ? 6 : 8;
    const int g = (nc + 3) >> 2;
    const int c0 = wv * g;
    const int c1 = c0 + g < nc ? c0 + g : nc;
    for (int cs = c0; cs < c1; cs += CW) {
        const int cnt = c1 - cs < CW ? c1 - cs : CW;
        double2 acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = mk(0, 0);
        const typename CT<T>::t* vp = V + (int64_t)cs * ldv;
        for (int64_t i = r0 + lane * R; i < r1; i += RW) {
            double2 xa[R], xb[R];
            IX::get(IX::ld(x0 + i), xa);
            if (NX > 1) IX::get(IX::ld(x1 + i), xb);
            typename IV::V vr[CW];
#pragma unroll
            for (int c = 0; c < CW; ++c)
                if (c < cnt) vr[c] = IV::ldnt(vp + (int64_t)c * ldv + i);
#pragma unroll
            for (int c = 0; c < CW; ++c)
                if (c < cnt) {
                    double2 v[R];
                    IV::get(vr[c], v);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        acc[c] = cadd(acc[c], cjmul(v[r], xa[r]));
                        if (NX > 1) acc[8 + c] = cadd(acc[8 + c], cjmul(v[r], xb[r]));
                    }
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

// k_shared_dot: gs_dot with one vector per member for members that all
// project on the same basis V. A block takes the row range of gs_dot's block
// for SHARED_MG members at once; its eight waves split the columns (at most 4
// each, so that 4 columns x 4 members fill the 16 accumulators of one
// reduce-scatter). Each basis row is read once per member group and each
// vector row once per wave from the caches. Rows are visited per lane in the
// same order and reduced by the same butterfly as in k_gs_dot, so the
// partial sums are identical; member b's values go to b's place in gs_dot's
// layout.
template <typename T, typename TX>
__global__ __launch_bounds__(512) void k_shared_dot(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int nc,
    const typename CT<TX>::t* __restrict__ x, int64_t x_ms, double2* __restrict__ partial,
    int nblk, int64_t n, int nmem, const int* __restrict__ act) {
    constexpr int MG = SHARED_MG;
    constexpr int CW = 16 / MG;
    using IV = RowIO<T, 1>;
    using IX = RowIO<TX, 1>;
    const int b0 = blockIdx.y * MG;
    bool on[MG];
    bool any = false;
#pragma unroll
    for (int m = 0; m < MG; ++m) {
        on[m] = b0 + m < nmem && (!act || act[b0 + m]);
        any = any || on[m];
    }
    if (!any) return;   // uniform over the block
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int NW = 8;
    const int64_t per = ((n + nblk - 1) / nblk + 63) / 64 * 64;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    const int nval = nc + 1;
    const int g = (nc + NW - 1) / NW;   // <= CW
    const int c0 = wv * g;
    const int cnt = nc - c0 < g ? nc - c0 : g;
    if (cnt > 0) {
        double2 acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = mk(0, 0);
        const typename CT<T>::t* vp = V + (int64_t)c0 * ldv;
        for (int64_t i = r0 + lane; i < r1; i += 64) {
            double2 xv[MG];
#pragma unroll
            for (int m = 0; m < MG; ++m) {
                xv[m] = mk(0, 0);
                if (on[m]) IX::get(IX::ld(x + (int64_t)(b0 + m) * x_ms + i), &xv[m]);
            }
#pragma unroll
            for (int c = 0; c < CW; ++c)
                if (c < cnt) {
                    double2 v;
                    IV::get(IV::ldnt(vp + (int64_t)c * ldv + i), &v);
#pragma unroll
                    for (int m = 0; m < MG; ++m) acc[m * CW + c] = cadd(acc[m * CW + c], cjmul(v, xv[m]));
                }
        }
        const double2 sum = rs16(acc, lane);
        if ((lane & 3) == 0) {
            const int q = (lane >> 2) & 15;
            const int m = q / CW, c = q % CW;
            if (c < cnt && on[m])
                partial[((int64_t)(b0 + m) * nval + c0 + c) * nblk + blockIdx.x] = sum;
        }
    }
    // ||x_b||^2, one wave per member, as gs_dot's last wave computes it
    if (wv < MG && on[wv]) {
        const typename CT<TX>::t* xl = x + (int64_t)(b0 + wv) * x_ms;
        double s2 = 0;
        for (int64_t i = r0 + lane; i < r1; i += 64) s2 += cabs2(to_d(xl[i]));
        s2 = wsum(s2);
        if (lane == 0) partial[((int64_t)(b0 + wv) * nval + nc) * nblk + blockIdx.x] = mk(s2, 0);
    }
}


// k_gs_update: one sweep forms NO outputs
//   y_o = sum_a beta[o][a] x_a - sum_{c<nc} V_c coef[o][c]
// with coefficients coef[mem*coef_ms + o*(MAXM+1) + c] and
// beta[mem*coef_ms + 2*(MAXM+1) + 2*o + a]. y_0 may alias x_0 (each row is
// read before it is written by the same thread).
template <typename T, int NX, int NO, int R>
__global__ __launch_bounds__(256) void k_gs_update(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int64_t v_ms, int nc,
    const typename CT<T>::t* x0, int64_t x0_ms, const typename CT<T>::t* __restrict__ x1,
    int64_t x1_ms, typename CT<T>::t* y0, int64_t y0_ms, typename CT<T>::t* __restrict__ y1,
    int64_t y1_ms, const double2* __restrict__ coef, int64_t coef_ms, int64_t n,
    const int* __restrict__ act) {
    using IO = RowIO<T, R>;
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
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * R; i < n;
         i += (int64_t)gridDim.x * blockDim.x * R) {
        double2 xa[R], xb[R], o0[R], o1[R];
        IO::get(IO::ld(x0 + i), xa);
        if (NX > 1) IO::get(IO::ld(x1 + i), xb);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            o0[r] = cmul(bt[0][0], xa[r]);
            o1[r] = mk(0, 0);
            if (NX > 1) o0[r] = cadd(o0[r], cmul(bt[0][1], xb[r]));
            if (NO > 1) o1[r] = cadd(cmul(bt[NO - 1][0], xa[r]), cmul(bt[NO - 1][1], xb[r]));
        }
        for (int cb = 0; cb < nc; cb += CH) {
            typename IO::V vr[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (cb + c < nc) vr[c] = IO::ldnt(V + (int64_t)(cb + c) * ldv + i);
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (cb + c < nc) {
                    double2 v[R];
                    IO::get(vr[c], v);
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        o0[r] = csub(o0[r], cmul(v[r], cf[0][cb + c]));
                        if (NO > 1) o1[r] = csub(o1[r], cmul(v[r], cf[NO - 1][cb + c]));
                    }
                }
        }
        IO::put(y0 + i, o0);
        if (NO > 1) IO::put(y1 + i, o1);
    }
}

template <typename T, typename TX>
void gs_dot(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
            const typename CT<TX>::t* x0, int64_t x0_ms, const typename CT<TX>::t* x1,
            int64_t x1_ms, double2* partial, int nblk, int64_t n, int nmem, hipStream_t st,
            const int* act) {
    dim3 grid(nblk, nmem), blk(256);
    constexpr bool f32 = std::is_same<T, float>::value && std::is_same<TX, float>::value;
    const bool r2 = f32 && pairable(n, {ldv, v_ms, x0_ms, x1 ? x1_ms : 0}, {V, x0, x1});
#define GS_DOT(NX, R)                                                                          \
    hipLaunchKernelGGL((k_gs_dot<T, TX, NX, R>), grid, blk, 0, st, V, ldv, v_ms, nc, x0, x0_ms, \
                       x1, x1_ms, partial, nblk, n, act)
    if (f32 && r2) {
        if (x1) GS_DOT(2, f32 ? 2 : 1);
        else GS_DOT(1, f32 ? 2 : 1);
    } else {
        if (x1) GS_DOT(2, 1);
        else GS_DOT(1, 1);
    }
#undef GS_DOT
}

template <typename T>
void gs_update(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
               const typename CT<T>::t* x0, int64_t x0_ms, const typename CT<T>::t* x1,
               int64_t x1_ms, typename CT<T>::t* y0, int64_t y0_ms, typename CT<T>::t* y1,
               int64_t y1_ms, const double2* coef, int64_t coef_ms, int64_t n, int nmem,
               hipStream_t st, const int* act) {
    constexpr bool f32 = std::is_same<T, float>::value;
    const bool r2 = f32 && pairable(n, {ldv, v_ms, x0_ms, x1 ? x1_ms : 0, y0_ms, y1 ? y1_ms : 0},
                                    {V, x0, x1, y0, y1});
    // tuned blocks per member (identical results: rows are independent)
    TuneScope ts("gs_update", sweep_shape(n, nmem, x1 ? 2 : 1, r2), SWEEP_NCAND, 0, st,
                 nc + (x1 ? 4 : 2));
    dim3 grid(sweep_nblk(n, nmem, f32, ts.choice()), nmem), blk(256);
#define GS_UPD(NX, R)                                                                            \
    hipLaunchKernelGGL((k_gs_update<T, NX, NX, R>), grid, blk, 0, st, V, ldv, v_ms, nc, x0, x0_ms, \
                       x1, x1_ms, y0, y0_ms, y1, y1_ms, coef, coef_ms, n, act)
    if (f32 && r2) {
        if (x1) GS_UPD(2, f32 ? 2 : 1);
        else GS_UPD(1, f32 ? 2 : 1);
    } else {
        if (x1) GS_UPD(2, 1);
        else GS_UPD(1, 1);
    }
#undef GS_UPD
}

// ---------------------------------------------------------------------------
// Block Gram-Schmidt sweeps of the s-step Arnoldi cycle: the same row
// partition and reductions as the DCGS2 sweeps, with NX (<= BLK_MAX) block
// vectors X_a = X + a*ldx in place of r_j and w.
// SECOND: the conditional second sweep pair of the s-step cycle (the same
// code under its own name, so that profiles keep the two pairs apart)
template <typename T, int NX, int R, bool SECOND>
__global__ __launch_bounds__(256) void k_blk_dot(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int64_t v_ms, int nc,
    const typename CT<T>::t* __restrict__ X, int64_t ldx, int64_t x_ms,
    double2* __restrict__ partial, int nblk, int64_t n, const int* __restrict__ act) {
    using IO = RowIO<T, R>;
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    X += mem * x_ms;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    constexpr int RW = 64 * R;
    const int64_t per = ((n + nblk - 1) / nblk + RW - 1) / RW * RW;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    const int nval = NX * nc;
    double2* pout = partial + (int64_t)mem * nval * nblk + blockIdx.x;
    // accumulators: CW columns x NX vectors <= 16 (one reduce-scatter)
    constexpr int CW = NX == 1 ? 8 : 16 / NX;
    const int g = (nc + 3) >> 2;
    const int c0 = wv * g;
    const int c1 = c0 + g < nc ? c0 + g : nc;
    for (int cs = c0; cs < c1; cs += CW) {
        const int cnt = c1 - cs < CW ? c1 - cs : CW;
        double2 acc[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[q] = mk(0, 0);
        const typename CT<T>::t* vp = V + (int64_t)cs * ldv;
        for (int64_t i = r0 + lane * R; i < r1; i += RW) {
            double2 xv[NX][R];
#pragma unroll
            for (int a = 0; a < NX; ++a) IO::get(IO::ld(X + (int64_t)a * ldx + i), xv[a]);
            typename IO::V vr[CW];
#pragma unroll
            for (int c = 0; c < CW; ++c)
                if (c < cnt) vr[c] = IO::ldnt(vp + (int64_t)c * ldv + i);
#pragma unroll
            for (int c = 0; c < CW; ++c)
                if (c < cnt) {
                    double2 v[R];
                    IO::get(vr[c], v);
#pragma unroll
                    for (int a = 0; a < NX; ++a)
#pragma unroll
                        for (int r = 0; r < R; ++r) acc[a * CW + c] = cadd(acc[a * CW + c], cjmul(v[r], xv[a][r]));
                }
        }
        const double2 sum = rs16(acc, lane);
        if ((lane & 3) == 0) {
            const int q = (lane >> 2) & 15;
            const int a = q / CW, c = q % CW;
            if (a < NX && c < cnt) pout[(int64_t)(a * nc + cs + c) * nblk] = sum;
        }
    }
}

template <typename T, int NB, int R, bool SECOND>
__global__ __launch_bounds__(256) void k_blk_update(
    const typename CT<T>::t* __restrict__ V, int64_t ldv, int64_t v_ms, int nc,
    typename CT<T>::t* X, int64_t ldx, int64_t x_ms, const double2* __restrict__ coef,
    int64_t coef_ms, int64_t n, const int* __restrict__ act) {
    using IO = RowIO<T, R>;
    constexpr int CH = std::is_same<T, float>::value ? 8 : 4;
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    X += mem * x_ms;
    coef += mem * coef_ms;
    __shared__ double2 cf[NB][MAXM + 1];
    __shared__ double2 bt[NB][NB];
    for (int t = threadIdx.x; t < NB * nc; t += blockDim.x) {
        const int o = t / nc, c = t % nc;
        cf[o][c] = coef[o * (MAXM + 1) + c];
    }
    if (threadIdx.x < NB * NB) {
        const int o = threadIdx.x / NB, a = threadIdx.x % NB;
        bt[o][a] = coef[BLK_MAX * (MAXM + 1) + o * BLK_MAX + a];
    }
    __syncthreads();
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * R; i < n;
         i += (int64_t)gridDim.x * blockDim.x * R) {
        double2 o[NB][R];
        {
            double2 xv[NB][R];
#pragma unroll
            for (int a = 0; a < NB; ++a) IO::get(IO::ld(X + (int64_t)a * ldx + i), xv[a]);
#pragma unroll
            for (int q = 0; q < NB; ++q)
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    double2 acc = mk(0, 0);
#pragma unroll
                    for (int a = 0; a < NB; ++a) acc = cadd(acc, cmul(bt[q][a], xv[a][r]));
                    o[q][r] = acc;
                }
        }
        for (int cb = 0; cb < nc; cb += CH) {
            typename IO::V vr[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (cb + c < nc) vr[c] = IO::ldnt(V + (int64_t)(cb + c) * ldv + i);
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (cb + c < nc) {
                    double2 v[R];
                    IO::get(vr[c], v);
#pragma unroll
                    for (int q = 0; q < NB; ++q)
#pragma unroll
                        for (int r = 0; r < R; ++r) o[q][r] = csub(o[q][r], cmul(v[r], cf[q][cb + c]));
                }
        }
#pragma unroll
        for (int q = 0; q < NB; ++q) IO::put(X + (int64_t)q * ldx + i, o[q]);
    }
}

// Blocks of 5..8 vectors (FP32 basis) on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64: A[i][k] from lane i + 16k, B[k][j] from lane
// j + 16k; register v of lane l holds D[l / 16 + 4v][l % 16]). With 16 FP64
// accumulators per lane the VALU sweeps above take two basis columns per
// pass at this width and re-read the block for every pair; the matrix cores
// keep the sums of all columns in 16 x 16 tiles spread over the wavefront,
// so every row of the basis and of the block is read once. Complex products
// are real ones over (real, imaginary) pairs: sum_k conj(v) x is
// (vr xr + vi xi) + i (vr xi - vi xr). The FP32 entries convert exactly, so
// the products are FP64 throughout, as in the VALU sweeps (sums in another
// order). n must be a multiple of 16 (16-row chunks).
typedef double d4v __attribute__((ext_vector_type(4)));
constexpr int B8_MT = (MAXM + 1 + 15) / 16;   // column tiles of a projection sweep

__device__ __forceinline__ d4v mfma64(double a, double b, d4v c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Projection sweep G[c][a] = sum_rows conj(V_c) X_a, c < nc, a < nx <= 8:
// M = basis columns (16 per tile), N = (a, re/im), K = (row, re/im). A
// wavefront takes 16-row chunks of its block's rows (lane group lg = lane / 16
// holds four rows of the chunk); the four wavefronts' tiles are summed
// in LDS into the block's partial sums (same layout as k_blk_dot).
template <bool SECOND>
__global__ __launch_bounds__(256, 4) void k_blk_dot8(const float2* __restrict__ V, int64_t ldv,
                                                  int64_t v_ms, int nc, const float2* __restrict__ X,
                                                  int64_t ldx, int64_t x_ms, int nx,
                                                  double2* __restrict__ partial, int nblk, int64_t n,
                                                  const int* __restrict__ act) {
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    X += mem * x_ms;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t per = ((n + nblk - 1) / nblk + 63) / 64 * 64;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    const int nmt = (nc + 15) >> 4;
    const int xa = li >> 1, xc = li & 1;   // block vector and part of this lane's N column
    const float2* xp = X + (int64_t)(xa < nx ? xa : 0) * ldx;
    d4v acc[B8_MT];
#pragma unroll
    for (int tm = 0; tm < B8_MT; ++tm) acc[tm] = d4v{0, 0, 0, 0};
    // loads of one 16-row chunk: the B operand (block entries) and the A
    // operands of the first NT column tiles
    auto load = [&](int64_t row0, double (&bop)[8], auto& vs, auto ntc) {
        constexpr int NT = decltype(ntc)::value;
        // rows of lane group lg: 2lg, 2lg+1 and 8+2lg, 9+2lg of the chunk, so
        // each 16-byte load of the four groups covers 64 contiguous bytes
        const int64_t ra = row0 + 2 * lg, rb8 = row0 + 8 + 2 * lg;
        f4v x01 = {0, 0, 0, 0}, x23 = {0, 0, 0, 0};
        if (xa < nx) {
            x01 = *(const f4v*)(xp + ra);
            x23 = *(const f4v*)(xp + rb8);
        }
        const float xs[8] = {x01.x, x01.y, x01.z, x01.w, x23.x, x23.y, x23.z, x23.w};
        // K entry (row t = u / 2, part u % 2) of N column (xa, xc)
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const float xr = xs[2 * (u >> 1)], xi = xs[2 * (u >> 1) + 1];
            bop[u] = (u & 1) == 0 ? (xc == 0 ? xr : xi) : (xc == 0 ? xi : -xr);
        }
#pragma unroll
        for (int tm = 0; tm < NT; ++tm) {
            const int c = tm * 16 + li;
            f4v v01 = {0, 0, 0, 0}, v23 = {0, 0, 0, 0};
            if (tm < nmt && c < nc) {
                const float2* vp = V + (int64_t)c * ldv;
                v01 = __builtin_nontemporal_load((const f4v*)(vp + ra));
                v23 = __builtin_nontemporal_load((const f4v*)(vp + rb8));
            }
            vs[tm][0] = v01.x;
            vs[tm][1] = v01.y;
            vs[tm][2] = v01.z;
            vs[tm][3] = v01.w;
            vs[tm][4] = v23.x;
            vs[tm][5] = v23.y;
            vs[tm][6] = v23.z;
            vs[tm][7] = v23.w;
        }
    };
    auto mma = [&](const double (&bop)[8], const auto& vs, auto ntc) {
        constexpr int NT = decltype(ntc)::value;
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int tm = 0; tm < NT; ++tm)
                if (tm < nmt) acc[tm] = mfma64(vs[tm][u], bop[u], acc[tm]);
    };
    if (nmt <= 2) {
        // one or two column tiles: a chunk holds few bytes per wavefront, so
        // two chunks (64 rows apart, this wavefront's next one) are loaded
        // before either's MFMAs; each accumulator takes its chunks in the
        // same order as below
        using N2 = std::integral_constant<int, 2>;
        for (int64_t row0 = r0 + 16 * wv; row0 < r1; row0 += 128) {
            const bool two = row0 + 64 < r1;   // uniform
            double bopA[8], bopB[8];
            float vsA[2][8], vsB[2][8];
            load(row0, bopA, vsA, N2{});
            load(two ? row0 + 64 : row0, bopB, vsB, N2{});
            mma(bopA, vsA, N2{});
            if (two) mma(bopB, vsB, N2{});
        }
    } else {
        using NM = std::integral_constant<int, B8_MT>;
        for (int64_t row0 = r0 + 16 * wv; row0 < r1; row0 += 64) {
            double bop[8];
            float vs[B8_MT][8];
            load(row0, bop, vs, NM{});
            mma(bop, vs, NM{});
        }
    }
    __shared__ double red[4][B8_MT][16][16];
#pragma unroll
    for (int tm = 0; tm < B8_MT; ++tm)
        if (tm < nmt)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wv][tm][lg + 4 * v][li] = acc[tm][v];
    __syncthreads();
    double2* pout = partial + (int64_t)mem * nx * nc * nblk + blockIdx.x;
    for (int e = threadIdx.x; e < nmt * 128; e += 256) {
        const int tm = e >> 7, i = (e >> 3) & 15, a = e & 7;
        const int c = tm * 16 + i;
        if (c < nc && a < nx) {
            double re = 0, im = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                re += red[w][tm][i][2 * a];
                im += red[w][tm][i][2 * a + 1];
            }
            pout[(int64_t)(a * nc + c) * nblk] = mk(re, im);
        }
    }
}

// Batched projection on one shared basis, G[c][b] = sum_rows conj(V_c) X_b
// for c < nc <= 32 (FP32 basis) and FP64 member vectors X_b, on the FP64
// matrix cores: M = basis columns (two tiles of 16), N = (member, re/im)
// with eight members per tile and two tiles per block, K = (row, re/im), in
// the 16-row chunks of k_blk_dot8. A block takes gs_dot's row range for 16
// members, so every basis row is read once for all of them (the VALU form
// reads it once per group of SHARED_MG members); ||X_b||^2 is summed on the
// VALU from the same loads. Partial sums in gs_dot's layout, column nc the
// squared norm. n must be a multiple of 16.
constexpr int SD8_MEM = 16;
static_assert(SHARED_NC_MAX <= 32, "k_shared_dot8 holds two column tiles");

__global__ __launch_bounds__(256) void k_shared_dot8(const float2* __restrict__ V, int64_t ldv,
                                                     int nc, const double2* __restrict__ X,
                                                     int64_t x_ms, double2* __restrict__ partial,
                                                     int nblk, int64_t n, int nmem,
                                                     const int* __restrict__ act) {
    const int g0 = blockIdx.y * SD8_MEM;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int xa = li >> 1, xc = li & 1;   // member (in its tile) and part of this lane's N column
    // per N tile: any member active (uniform), its first active member, and
    // this lane's member; an inactive lane reads the first active member's
    // rows (same cache lines as that lane) and uses zeros
    bool ton[2], mon[2];
    const double2* xp[2];
    bool any = false;
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
        int first = -1;
        for (int a = 7; a >= 0; --a) {
            const int m = g0 + tn * 8 + a;
            if (m < nmem && (!act || act[m])) first = m;
        }
        ton[tn] = first >= 0;
        any = any || ton[tn];
        const int m = g0 + tn * 8 + xa;
        mon[tn] = m < nmem && (!act || act[m]);
        xp[tn] = X + (int64_t)(mon[tn] ? m : (first >= 0 ? first : g0)) * x_ms;
    }
    if (!any) return;   // uniform over the block
    const int64_t per = ((n + nblk - 1) / nblk + 63) / 64 * 64;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = r0 + per < n ? r0 + per : n;
    const int nmt = (nc + 15) >> 4;
    d4v acc[2][2];
#pragma unroll
    for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) acc[tm][tn] = d4v{0, 0, 0, 0};
    double s2[2] = {0, 0};
    for (int64_t row0 = r0 + 16 * wv; row0 < r1; row0 += 64) {
        // rows of lane group lg: 2lg, 2lg+1, 8+2lg, 9+2lg of the chunk
        const int64_t ra = row0 + 2 * lg, rb8 = row0 + 8 + 2 * lg;
        double bop[2][8];   // K entry (row u / 2, part u % 2) of N column (xa, xc)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
#pragma unroll
            for (int u = 0; u < 8; ++u) bop[tn][u] = 0;
            if (ton[tn]) {
                const double2* p = xp[tn];
                double2 xv[4] = {p[ra], p[ra + 1], p[rb8], p[rb8 + 1]};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    xv[t] = csel(mon[tn], xv[t], mk(0, 0));
                    s2[tn] += xc == 0 ? xv[t].x * xv[t].x + xv[t].y * xv[t].y : 0.0;
                    bop[tn][2 * t] = xc == 0 ? xv[t].x : xv[t].y;
                    bop[tn][2 * t + 1] = xc == 0 ? xv[t].y : -xv[t].x;
                }
            }
        }
        float vs[2][8];
#pragma unroll
        for (int tm = 0; tm < 2; ++tm) {
            const int c = tm * 16 + li;
            f4v v01 = {0, 0, 0, 0}, v23 = {0, 0, 0, 0};
            if (tm < nmt) {
                const float2* vp = V + (int64_t)(c < nc ? c : 0) * ldv;
                v01 = __builtin_nontemporal_load((const f4v*)(vp + ra));
                v23 = __builtin_nontemporal_load((const f4v*)(vp + rb8));
                if (c >= nc) {
                    v01 = f4v{0, 0, 0, 0};
                    v23 = f4v{0, 0, 0, 0};
                }
            }
            vs[tm][0] = v01.x;
            vs[tm][1] = v01.y;
            vs[tm][2] = v01.z;
            vs[tm][3] = v01.w;
            vs[tm][4] = v23.x;
            vs[tm][5] = v23.y;
            vs[tm][6] = v23.z;
            vs[tm][7] = v23.w;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int tm = 0; tm < 2; ++tm)
                if (tm < nmt)
#pragma unroll
                    for (int tn = 0; tn < 2; ++tn)
                        if (ton[tn]) acc[tm][tn] = mfma64(vs[tm][u], bop[tn][u], acc[tm][tn]);
    }
    __shared__ double red[4][2][2][16][16];
    __shared__ double nrm[4][4][SD8_MEM];
#pragma unroll
    for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn)
#pragma unroll
            for (int v = 0; v < 4; ++v) red[wv][tm][tn][lg + 4 * v][li] = acc[tm][tn][v];
    if (xc == 0) {
        nrm[wv][lg][xa] = s2[0];
        nrm[wv][lg][8 + xa] = s2[1];
    }
    __syncthreads();
    const int nval = nc + 1;
    for (int e = threadIdx.x; e < nmt * 16 * SD8_MEM; e += 256) {
        const int tm = e / (16 * SD8_MEM), i = (e / SD8_MEM) & 15, ml = e % SD8_MEM;
        const int c = tm * 16 + i, m = g0 + ml;
        if (c < nc && m < nmem && (!act || act[m])) {
            double re = 0, im = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                re += red[w][tm][ml >> 3][i][2 * (ml & 7)];
                im += red[w][tm][ml >> 3][i][2 * (ml & 7) + 1];
            }
            partial[((int64_t)m * nval + c) * nblk + blockIdx.x] = mk(re, im);
        }
    }
    if (threadIdx.x < SD8_MEM) {
        const int m = g0 + threadIdx.x;
        if (m < nmem && (!act || act[m])) {
            double t = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w)
#pragma unroll
                for (int g = 0; g < 4; ++g) t += nrm[w][g][threadIdx.x];
            partial[((int64_t)m * nval + nc) * nblk + blockIdx.x] = mk(t, 0);
        }
    }
}

template <typename T, typename TX>
void shared_dot(const typename CT<T>::t* V, int64_t ldv, int nc, const typename CT<TX>::t* x,
                int64_t x_ms, double2* partial, int nblk, int64_t n, int nmem, hipStream_t st,
                const int* act) {
    if (nc < 1 || nc > SHARED_NC_MAX) throw std::invalid_argument("shared_dot: nc out of range");
    if constexpr (std::is_same<T, float>::value && std::is_same<TX, double>::value) {
        if (n % 16 == 0) {   // FP32 basis, FP64 members: the matrix-core form
            dim3 grid(nblk, (nmem + SD8_MEM - 1) / SD8_MEM), blk(256);
            hipLaunchKernelGGL(k_shared_dot8, grid, blk, 0, st, V, ldv, nc, x, x_ms, partial, nblk,
                               n, nmem, act);
            return;
        }
    }
    dim3 grid(nblk, (nmem + SHARED_MG - 1) / SHARED_MG), blk(512);
    hipLaunchKernelGGL((k_shared_dot<T, TX>), grid, blk, 0, st, V, ldv, nc, x, x_ms, partial,
                       nblk, n, nmem, act);
}

template void shared_dot<float, double>(const float2*, int64_t, int, const double2*, int64_t,
                                        double2*, int, int64_t, int, hipStream_t, const int*);
template void shared_dot<double, double>(const double2*, int64_t, int, const double2*, int64_t,
                                         double2*, int, int64_t, int, hipStream_t, const int*);

// Update sweep X_q <- sum_a bt[q][a] X_a - sum_c V_c cf[q][c], q < nx <= 8
// (coefficients as in k_blk_update): M = outputs (q, re/im), N = rows (16 per
// tile), K = (input, re/im) over the inputs V_0..V_{nc-1}, X_0..X_{nx-1}. An
// MFMA pair (t, p) takes inputs 4t..4t+3 (lane group lg = lane / 16 supplies
// input 4t + lg) with their real parts (p = 0) and imaginary parts (p = 1), so
// a lane loads whole complex entries and feeds each to two MFMAs. The
// coefficient operand of lane position l and pair (t, p) is the same in every
// wavefront: staged once per block in LDS. A wavefront takes four 16-row tiles
// at a time. Lane l ends with output lg + 4v of row l % 16: lanes of even and
// odd lg pair up into complex results, stored as 128-byte runs per column.
constexpr int B8_T2 = (MAXM + 1 + 8 + 3) / 4;   // input quads of an update sweep
template <bool SECOND>
__global__ __launch_bounds__(256) void k_blk_update8(const float2* __restrict__ V, int64_t ldv,
                                                     int64_t v_ms, int nc, float2* X, int64_t ldx,
                                                     int64_t x_ms, int nx,
                                                     const double2* __restrict__ coef,
                                                     int64_t coef_ms, int64_t n,
                                                     const int* __restrict__ act) {
    const int mem = blockIdx.y;
    if (act && !act[mem]) return;
    V += mem * v_ms;
    X += mem * x_ms;
    coef += mem * coef_ms;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int nin = nc + nx, T2 = (nin + 3) >> 2;
    __shared__ double aop[B8_T2][2][64];
    for (int e = threadIdx.x; e < T2 * 128; e += 256) {
        const int t = e >> 7, pt = (e >> 6) & 1, l = e & 63;
        const int q = (l & 15) >> 1, comp = l & 1, inp = 4 * t + (l >> 4);
        double2 w = mk(0, 0);
        if (q < nx && inp < nin)
            w = inp < nc ? cscale(coef[q * (MAXM + 1) + inp], -1.0)
                         : coef[BLK_MAX * (MAXM + 1) + q * BLK_MAX + (inp - nc)];
        aop[t][pt][l] = comp == 0 ? (pt == 0 ? w.x : -w.y) : (pt == 0 ? w.y : w.x);
    }
    __syncthreads();
    for (int64_t rb = ((int64_t)blockIdx.x * 4 + wv) * 64; rb < n; rb += (int64_t)gridDim.x * 256) {
        d4v d[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) d[rt] = d4v{0, 0, 0, 0};
        // rows of this lane in the four tiles (those past n, in the last
        // chunk, read row n - 16 + li and are not stored)
        int64_t rows[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
            const int64_t row = rb + rt * 16 + li;
            rows[rt] = row < n ? row : n - 16 + li;
        }
        // two input quads per round (four measured 2 % slower: two waves per
        // SIMD instead of four): every load issued before the MFMAs, none in a
        // branch (an input past the last reads column 0 with coefficient 0)
        for (int t0 = 0; t0 < T2; t0 += 2) {
            float2 xv[2][4];
            double a0[2], a1[2];
#pragma unroll
            for (int tt = 0; tt < 2; ++tt) {
                const int t = t0 + tt;
                const int inp = 4 * t + lg;
                const bool on = t < T2 && inp < nin;
                const float2* col = !on ? V : inp < nc ? V + (int64_t)inp * ldv : X + (int64_t)(inp - nc) * ldx;
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) xv[tt][rt] = col[rows[rt]];
                const int ts = t < B8_T2 ? t : B8_T2 - 1;
                a0[tt] = t < T2 ? aop[ts][0][lane] : 0.0;
                a1[tt] = t < T2 ? aop[ts][1][lane] : 0.0;
            }
#pragma unroll
            for (int tt = 0; tt < 2; ++tt)
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) {
                    d[rt] = mfma64(a0[tt], xv[tt][rt].x, d[rt]);
                    d[rt] = mfma64(a1[tt], xv[tt][rt].y, d[rt]);
                }
        }
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double im = __shfl_down(d[rt][v], 16, 64);
                const int qo = (lg >> 1) + 2 * v;
                const int64_t row = rb + rt * 16 + li;
                if ((lg & 1) == 0 && qo < nx && row < n)
                    X[(int64_t)qo * ldx + row] = make_float2((float)d[rt][v], (float)im);
            }
    }
}

template <typename T>
void blk_dot(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
             const typename CT<T>::t* X, int64_t ldx, int64_t x_ms, int nx, double2* partial,
             int nblk, int64_t n, int nmem, hipStream_t st, const int* act, bool second) {
    dim3 grid(nblk, nmem), blk(256);
    constexpr bool f32 = std::is_same<T, float>::value;
    if (nx > 4) {
        if (!f32 || n % 16 != 0 || nx > 8 || (nc + 15) / 16 > B8_MT)
            throw std::runtime_error("blk_dot: blocks of 5..8 need FP32, n % 16 == 0 and nc <= MAXM + 1");
        const float2* Vf = (const float2*)V;
        const float2* Xf = (const float2*)X;
        if (second)
            hipLaunchKernelGGL(k_blk_dot8<true>, grid, blk, 0, st, Vf, ldv, v_ms, nc, Xf, ldx, x_ms, nx,
                               partial, nblk, n, act);
        else
            hipLaunchKernelGGL(k_blk_dot8<false>, grid, blk, 0, st, Vf, ldv, v_ms, nc, Xf, ldx, x_ms, nx,
                               partial, nblk, n, act);
        return;
    }
    const bool r2 = f32 && pairable(n, {ldv, v_ms, ldx, x_ms}, {V, X});
#define BLK_DOT(NX, R)                                                                          \
    do {                                                                                        \
        if (second)                                                                             \
            hipLaunchKernelGGL((k_blk_dot<T, NX, R, true>), grid, blk, 0, st, V, ldv, v_ms, nc, X, \
                               ldx, x_ms, partial, nblk, n, act);                               \
        else                                                                                    \
            hipLaunchKernelGGL((k_blk_dot<T, NX, R, false>), grid, blk, 0, st, V, ldv, v_ms, nc, \
                               X, ldx, x_ms, partial, nblk, n, act);                            \
    } while (0)
#define BLK_DOT_R(R)                  \
    switch (nx) {                     \
        case 1: BLK_DOT(1, R); break; \
        case 2: BLK_DOT(2, R); break; \
        case 3: BLK_DOT(3, R); break; \
        default: BLK_DOT(4, R); break; \
    }
    if (r2) {
        BLK_DOT_R(f32 ? 2 : 1)
    } else {
        BLK_DOT_R(1)
    }
#undef BLK_DOT_R
#undef BLK_DOT
}

template <typename T>
void blk_update(const typename CT<T>::t* V, int64_t ldv, int64_t v_ms, int nc,
                typename CT<T>::t* X, int64_t ldx, int64_t x_ms, int nx, const double2* coef,
                int64_t coef_ms, int64_t n, int nmem, hipStream_t st, const int* act, bool second) {
    constexpr bool f32 = std::is_same<T, float>::value;
    const bool r2 = f32 && pairable(n, {ldv, v_ms, ldx, x_ms}, {V, X});
    // tuned blocks per member (identical results: rows are independent)
    TuneScope ts("blk_update", sweep_shape(n, nmem, nx, r2), SWEEP_NCAND, 0, st, nc + 2 * nx);
    dim3 grid(sweep_nblk(n, nmem, f32, ts.choice()), nmem), blk(256);
    if (nx > 4) {
        if (!f32 || n % 16 != 0 || nx > 8 || (nc + nx + 3) / 4 > B8_T2)
            throw std::runtime_error("blk_update: blocks of 5..8 need FP32, n % 16 == 0 and nc <= MAXM");
        const float2* Vf = (const float2*)V;
        float2* Xf = (float2*)X;
        if (second)
            hipLaunchKernelGGL(k_blk_update8<true>, grid, blk, 0, st, Vf, ldv, v_ms, nc, Xf, ldx, x_ms, nx,
                               coef, coef_ms, n, act);
        else
            hipLaunchKernelGGL(k_blk_update8<false>, grid, blk, 0, st, Vf, ldv, v_ms, nc, Xf, ldx, x_ms, nx,
                               coef, coef_ms, n, act);
        return;
    }
#define BLK_UPD(NB, R)                                                                         \
    do {                                                                                       \
        if (second)                                                                            \
            hipLaunchKernelGGL((k_blk_update<T, NB, R, true>), grid, blk, 0, st, V, ldv, v_ms, nc, \
                               X, ldx, x_ms, coef, coef_ms, n, act);                           \
        else                                                                                   \
            hipLaunchKernelGGL((k_blk_update<T, NB, R, false>), grid, blk, 0, st, V, ldv, v_ms, \
                               nc, X, ldx, x_ms, coef, coef_ms, n, act);                       \
    } while (0)
#define BLK_UPD_R(R)                  \
    switch (nx) {                     \
        case 1: BLK_UPD(1, R); break; \
        case 2: BLK_UPD(2, R); break; \
        case 3: BLK_UPD(3, R); break; \
        default: BLK_UPD(4, R); break; \
    }
    if (r2) {
        BLK_UPD_R(f32 ? 2 : 1)
    } else {
        BLK_UPD_R(1)
    }
#undef BLK_UPD_R
#undef BLK_UPD
}

template void blk_dot<float>(const float2*, int64_t, int64_t, int, const float2*, int64_t, int64_t,
                             int, double2*, int, int64_t, int, hipStream_t, const int*, bool);
template void blk_update<float>(const float2*, int64_t, int64_t, int, float2*, int64_t, int64_t,
                                int, const double2*, int64_t, int64_t, int, hipStream_t,
                                const int*, bool);


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

static int vec_grid(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (int)(g > 8192 ? 8192 : g);
}

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
// out_s = keep_s * out_s + sum_l V_l coef[l + s*ldc], summed from out_s
// (if kept) in the order of l.
//
// The coefficients are the same for every row, so they are read with uniform
// (scalar) loads straight from `coef` and enter the multiply-adds as scalar
// operands; each complex multiply-add is four FP64 fused multiply-adds. MO is
// the number of outputs a launch computes: nout itself up to 8 (no output
// computed in vain), else VC_MAXOUT, where outputs nout..MO-1 repeat output 0
// (same coefficients, same store).
constexpr int VC_MAXOUT = MAXNS + 2;

// acc += v * w, real and imaginary parts each by two fused multiply-adds
static __device__ __forceinline__ void cmac(double2& acc, double2 v, double2 w) {
    acc.x = fma(v.x, w.x, acc.x);
    acc.x = fma(-v.y, w.y, acc.x);
    acc.y = fma(v.x, w.y, acc.y);
    acc.y = fma(v.y, w.x, acc.y);
}

template <typename T, int R, int MO>
__global__ __launch_bounds__(256) void k_vcombine(const typename CT<T>::t* __restrict__ V,
                                                  int64_t ldv, int64_t v_ms, int ncols,
                                                  const double2* __restrict__ coef, int ldc,
                                                  int64_t c_ms, int nout, double2* __restrict__ out,
                                                  int64_t o_stride, int64_t o_ms, unsigned keep,
                                                  int64_t n, const int* __restrict__ act) {
    using IO = RowIO<T, R>;
    constexpr int CH = 8;   // basis columns loaded per batch (loads in flight per lane)
    const int b = blockIdx.y;
    if (act && !act[b]) return;
    V += b * v_ms;
    coef += b * c_ms;
    out += b * o_ms;
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * R; i < n;
         i += (int64_t)gridDim.x * blockDim.x * R) {
        // A kept output starts its sum, loaded first (the loads' latency
        // overlaps the basis loads); an output not kept loads output 0 and
        // drops it, so no load sits in a branch of its own.
        double2 acc[MO][R];
#pragma unroll
        for (int s = 0; s < MO; ++s) {
            const bool kp = s < nout && ((keep >> s) & 1u);
            const double2* os = out + (kp ? s : 0) * o_stride;
#pragma unroll
            for (int r = 0; r < R; ++r) acc[s][r] = csel(kp, *at32(os, i + r), mk(0, 0));
        }
        for (int l0 = 0; l0 < ncols; l0 += CH) {
            typename IO::V vr[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (l0 + c < ncols) vr[c] = IO::ldnt(at32(V + (int64_t)(l0 + c) * ldv, i));
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (l0 + c < ncols) {
                    double2 v[R];
                    IO::get(vr[c], v);
#pragma unroll
                    for (int s = 0; s < MO; ++s) {
                        const double2 w = coef[l0 + c + (s < nout ? s : 0) * ldc];
#pragma unroll
                        for (int r = 0; r < R; ++r) cmac(acc[s][r], v[r], w);
                    }
                }
        }
        // outputs nout..MO-1 repeat the store of output 0 (same address, same
        // value): the stores run with no branch between them
#pragma unroll
        for (int s = 0; s < MO; ++s) {
            const bool real = s < nout;
            double2* os = out + (real ? s : 0) * o_stride;
#pragma unroll
            for (int r = 0; r < R; ++r) *at32(os, i + r) = csel(real, acc[s][r], acc[0][r]);
        }
    }
}

// The same combination when all members share one basis (v_ms = 0, the
// deflation basis of the projection step): a block takes MG members, so
// each basis row is read once for all of them. One row per lane (8-byte FP32
// loads). Per row and output the sum starts from the kept output and runs
// over l in the same order, with the same operations, as in k_vcombine.
// Members past nmem take member b0's coefficients and store nothing.
template <typename T, int MO, int MG>
__global__ __launch_bounds__(256) void k_vcombine2(const typename CT<T>::t* __restrict__ V,
                                                   int64_t ldv, int ncols,
                                                   const double2* __restrict__ coef, int ldc,
                                                   int64_t c_ms, int nout, double2* __restrict__ out,
                                                   int64_t o_stride, int64_t o_ms, unsigned keep,
                                                   int64_t n, int nmem, const int* __restrict__ act) {
    using IO = RowIO<T, 1>;
    constexpr int CH = 8;
    const int b0 = blockIdx.y * MG;
    bool on[MG];
    bool any = false;
#pragma unroll
    for (int m = 0; m < MG; ++m) {
        on[m] = b0 + m < nmem && (!act || act[b0 + m]);
        any = any || on[m];
    }
    if (!any) return;   // uniform over the block
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double2 acc[MG][MO];
#pragma unroll
        for (int m = 0; m < MG; ++m)
#pragma unroll
            for (int s = 0; s < MO; ++s) {
                const bool kp = on[m] && s < nout && ((keep >> s) & 1u);
                const double2 o = *at32(out + (int64_t)b0 * o_ms + (kp ? m * o_ms + s * o_stride : 0), i);
                acc[m][s] = csel(kp, o, mk(0, 0));
            }
        for (int l0 = 0; l0 < ncols; l0 += CH) {
            typename IO::V vr[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (l0 + c < ncols) vr[c] = IO::ldnt(at32(V + (int64_t)(l0 + c) * ldv, i));
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (l0 + c < ncols) {
                    double2 v;
                    IO::get(vr[c], &v);
#pragma unroll
                    for (int m = 0; m < MG; ++m) {
                        const double2* cm = coef + (int64_t)(b0 + m < nmem ? b0 + m : b0) * c_ms;
#pragma unroll
                        for (int s = 0; s < MO; ++s)
                            cmac(acc[m][s], v, cm[l0 + c + (s < nout ? s : 0) * ldc]);
                    }
                }
        }
        // per member, outputs nout..MO-1 repeat the store of output 0, as in
        // k_vcombine
#pragma unroll
        for (int m = 0; m < MG; ++m) {
            if (!on[m]) continue;
#pragma unroll
            for (int s = 0; s < MO; ++s) {
                const bool real = s < nout;
                *at32(out + (int64_t)(b0 + m) * o_ms + (real ? s : 0) * o_stride, i) =
                    csel(real, acc[m][s], acc[m][0]);
            }
        }
    }
}

template <typename T>
void vcombine(const typename CT<T>::t* V, int64_t ldv, int64_t v_mstride, int ncols,
              const double2* coef, int ldc, int64_t c_mstride, int nout, double2* out,
              int64_t o_stride, int64_t o_mstride, unsigned keep_mask, int64_t n, int nmem,
              hipStream_t st, const int* act) {
    constexpr bool f32 = std::is_same<T, float>::value;
    if (nout < 1 || nout > VC_MAXOUT) throw std::runtime_error("vcombine: output count out of range");
    if (n > AT32_ROWS) {   // rows are independent: launches of at most AT32_ROWS rows
        for (int64_t r0 = 0; r0 < n; r0 += AT32_ROWS)
            vcombine<T>(V + r0, ldv, v_mstride, ncols, coef, ldc, c_mstride, nout, out + r0, o_stride,
                        o_mstride, keep_mask, std::min(AT32_ROWS, n - r0), nmem, st, act);
        return;
    }
    if (v_mstride == 0 && nmem > 1 && nout <= 8) {
        // one shared basis: four members per block for up to 4 outputs, two
        // for more (the accumulators of MG x MO outputs stay in registers)
#define VCOMB2(MO, MG)                                                                           \
    hipLaunchKernelGGL((k_vcombine2<T, MO, MG>), dim3(vec_grid(n), (nmem + MG - 1) / MG),      \
                       dim3(256), 0, st, V, ldv, ncols, coef, ldc, c_mstride, nout, out, o_stride, \
                       o_mstride, keep_mask, n, nmem, act)
        switch (nout) {
            case 1: VCOMB2(1, 8); break;
            case 2: VCOMB2(2, 8); break;
            case 3: VCOMB2(3, 4); break;
            case 4: VCOMB2(4, 4); break;
            case 5: VCOMB2(5, 4); break;
            case 6: VCOMB2(6, 4); break;
            case 7: VCOMB2(7, 4); break;
            default: VCOMB2(8, 4); break;
        }
#undef VCOMB2
        return;
    }
    const bool r2 = f32 && pairable(n, {ldv, v_mstride}, {V});
    // tuned grid (identical results: rows are independent)
    TuneScope ts("vcombine", sweep_shape(n, nmem, nout, r2), 4, 0, st, ncols + nout);
    static const int gcap[4] = {8192, 2048, 4096, 16384};
    int64_t gx = (n + 255) / 256;
    if (gx > gcap[ts.choice()]) gx = gcap[ts.choice()];
    const dim3 grid((unsigned)gx, nmem), blk(256);
#define VCOMB(R, MO)                                                                            \
    hipLaunchKernelGGL((k_vcombine<T, R, MO>), grid, blk, 0, st, V, ldv, v_mstride, ncols, coef, \
                       ldc, c_mstride, nout, out, o_stride, o_mstride, keep_mask, n, act)
#define VCOMB_ALL(R)                          \
    switch (nout) {                           \
        case 1: VCOMB(R, 1); break;           \
        case 2: VCOMB(R, 2); break;           \
        case 3: VCOMB(R, 3); break;           \
        case 4: VCOMB(R, 4); break;           \
        case 5: VCOMB(R, 5); break;           \
        case 6: VCOMB(R, 6); break;           \
        case 7: VCOMB(R, 7); break;           \
        case 8: VCOMB(R, 8); break;           \
        default: VCOMB(1, VC_MAXOUT); break;  \
    }
    // accumulators sized for the outputs at hand (r = V s and up to 16 shifts)
    if (r2) {
        VCOMB_ALL(f32 ? 2 : 1)
    } else {
        VCOMB_ALL(1)
    }
#undef VCOMB_ALL
#undef VCOMB
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

// FP32 recombination on the matrix cores. The complex product W = V P is the
// real product W' = V' P' with V' = [Re V, Im V] and the 2x2 real blocks of
// P, and it is computed transposed, C = P'^T V'^T, with
// v_mfma_f32_16x16x4f32: per instruction a wavefront multiplies a 16 x 4
// block of P'^T (16 real outputs = 8 complex columns of W) by a 4 x 16 block
// of V'^T (16 consecutive rows). Lane l provides A[n = l % 16][k = l / 16]
// and B[k = l / 16][row = l % 16], and receives C[4 (l / 16) + r][row =
// l % 16], r = 0..3: the real and imaginary parts of two complex outputs of
// one row, so each lane stores two float2 and 16 lanes store 128 contiguous
// bytes of one output column. The contraction index is taken in quads of four
// complex basis columns: lane group g = l / 16 loads the whole complex entry
// (8 bytes) of column 4q + g at its row and feeds its real part to one
// instruction and its imaginary part to the next, whose A blocks hold the
// matching rows of P'^T (the k index runs over (quad, part, column in quad)).
// P'^T sits in LDS, padded to whole quads; a wavefront keeps S strips of 16
// rows in flight, NT n-tiles of 16 real outputs each (nout <= 8 NT), and loads
// the basis entries one group of U quads ahead.
// FP32 products accumulated in FP32, as in the VALU kernel.
typedef float mf4 __attribute__((ext_vector_type(4)));
constexpr int VRC_S = 2;   // strips of 16 rows per wavefront
constexpr int VRC_U = 4;   // quads (8 k-steps) per load group

template <int S, int NT, int U = 4>
__global__ __launch_bounds__(256) void k_vrecombine_mfma(const float2* __restrict__ V, int64_t ldv,
                                                         int ncols, const double2* __restrict__ P,
                                                         int ldp, int nout, float2* __restrict__ W,
                                                         int64_t ldw, int64_t n) {
    const int nq = (ncols + 3) / 4;             // quads of complex basis columns
    constexpr int np = NT * 16;
    const int kp = nq * 8;                      // real k entries: (quad, part, column in quad)
    extern __shared__ float at[];               // kp x np floats
    // A = P'^T: A[nn][k] with nn = 16 tt + i at at[(k * 16 + i) * NT + tt], so
    // that a lane reads its NT n-tiles' values contiguously; nn = 2j + q
    // (output j, real/imag), k = (qd * 2 + pp) * 4 + g for basis column
    // c = 4 qd + g, part pp
    for (int t = threadIdx.x; t < kp * np; t += blockDim.x) {
        const int k = t / np, nn = t % np;
        const int idx = (k * 16 + (nn & 15)) * NT + (nn >> 4);
        const int g = k & 3, pp = (k >> 2) & 1, qd = k >> 3;
        const int c = 4 * qd + g, j = nn >> 1, q = nn & 1;
        float v = 0;
        if (c < ncols && j < nout) {
            const double2 pv = P[c + (int64_t)j * ldp];
            v = q == 0 ? (pp == 0 ? (float)pv.x : -(float)pv.y) : (pp == 0 ? (float)pv.y : (float)pv.x);
        }
        at[idx] = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;   // row / n within a block, column within a quad
    const int64_t nstrip = (n + 15) / 16;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t nwave = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t s0 = wave * S; s0 < nstrip; s0 += nwave * S) {
        mf4 acc[S][NT];
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[s][t] = mf4{0, 0, 0, 0};
        // quads in groups of U: the basis entries of the next group are loaded
        // while the matrix cores work on the current one (two register
        // buffers, the group loop unrolled by two)
        auto load_g = [&](int g0, float2 (&b)[U][S]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = 4 * (g0 * U + u) + lk;   // complex basis column of this lane
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const int64_t row = (s0 + s) * 16 + lr;
                    f2v v{0.f, 0.f};
                    if (c < ncols && row < n) v = __builtin_nontemporal_load((const f2v*)(V + c * ldv + row));
                    b[u][s] = make_float2(v.x, v.y);
                }
            }
        };
        auto mma_g = [&](int g0, const float2 (&b)[U][S]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int qd = g0 * U + u;
                if (qd >= nq) break;
                const float* ar = at + ((qd * 8 + lk) * 16 + lr) * NT;   // real parts' rows
                const float* ai = ar + 4 * 16 * NT;                       // imaginary parts' rows
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const float a0 = ar[t], a1 = ai[t];
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b[u][s].x, acc[s][t], 0, 0, 0);
                        acc[s][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b[u][s].y, acc[s][t], 0, 0, 0);
                    }
                }
            }
        };
        const int ng = (nq + U - 1) / U;
        float2 ba[U][S], bb[U][S];
        load_g(0, ba);
        for (int g0 = 0; g0 < ng; g0 += 2) {
            if (g0 + 1 < ng) load_g(g0 + 1, bb);
            mma_g(g0, ba);
            if (g0 + 1 < ng) {
                if (g0 + 2 < ng) load_g(g0 + 2, ba);
                mma_g(g0 + 1, bb);
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t row = (s0 + s) * 16 + lr;
            if (row >= n) continue;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                // C rows 4 lk + r of n-tile t: outputs j = 8 t + 2 lk (r = 0, 1) and + 1 (r = 2, 3)
                const int j = 8 * t + 2 * lk;
                if (j < nout) W[(int64_t)j * ldw + row] = make_float2(acc[s][t][0], acc[s][t][1]);
                if (j + 1 < nout) W[(int64_t)(j + 1) * ldw + row] = make_float2(acc[s][t][2], acc[s][t][3]);
            }
        }
    }
}

template <typename T>
void vrecombine(const typename CT<T>::t* V, int64_t ldv, int ncols, const double2* P, int ldp,
                int nout, typename CT<T>::t* W, int64_t ldw, int64_t n, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
        const int nt = (2 * nout + 15) / 16;
        const size_t lds = (size_t)((ncols + 3) / 4) * 8 * nt * 16 * sizeof(float);
        if (ncols >= 1 && ncols <= MAXM + 1 && nout >= 1 && nout <= MAXM && lds <= 65536) {
            // enough strips for every CU: 4 waves per block, VRC_S strips of 16 rows per
            // wave, at most 2048 blocks looping over the rest (1.32 ms on the
            // 24^3x48 restart, 61 columns to 21: 0.49 of HBM; the VALU kernel 2.8 ms)
            // tuned (identical results: every output sums its k entries in the
            // same order): strips per wavefront and quads per load group
            char shape[64];
            std::snprintf(shape, sizeof shape, "%lld|%d|%d", (long long)n, ncols, nout);
            TuneScope ts("vrecombine_mfma", shape, 3, 0, st);
            const int S = ts.choice() == 1 ? 4 : ts.choice() == 2 ? 1 : VRC_S;
            const int64_t blocks = (n + 64 * S - 1) / (64 * S);
            const int grid = (int)(blocks > 2048 ? 2048 : (blocks < 1 ? 1 : blocks));
#define VRC_MFMA1(S_, NT, U_)                                                                 \
    hipLaunchKernelGGL((k_vrecombine_mfma<S_, NT, U_>), dim3(grid), dim3(256), lds, st, V, ldv, \
                       ncols, P, ldp, nout, W, ldw, n)
#define VRC_MFMA(NT)                                             \
    do {                                                         \
        if (ts.choice() == 1) VRC_MFMA1(4, NT, 2);               \
        else if (ts.choice() == 2) VRC_MFMA1(1, NT, 8);          \
        else VRC_MFMA1(VRC_S, NT, VRC_U);                        \
    } while (0)
            switch (nt) {
                case 1: VRC_MFMA(1); break;
                case 2: VRC_MFMA(2); break;
                case 3: VRC_MFMA(3); break;
                case 4: VRC_MFMA(4); break;
                case 5: VRC_MFMA(5); break;
                case 6: VRC_MFMA(6); break;
                case 7: VRC_MFMA(7); break;
                default: VRC_MFMA(8); break;
            }
#undef VRC_MFMA
#undef VRC_MFMA1
            return;
        }
    }
    constexpr int CH = std::is_same<T, float>::value ? 32 : 16;
    hipLaunchKernelGGL((k_vrecombine<T, CH>), dim3(vec_grid(n)), dim3(256), 0, st, V, ldv, ncols,
                       P, ldp, nout, W, ldw, n);
}
template void vrecombine<double>(const double2*, int64_t, int, const double2*, int, int, double2*,
                                 int64_t, int64_t, hipStream_t);
template void vrecombine<float>(const float2*, int64_t, int, const double2*, int, int, float2*,
                                int64_t, int64_t, hipStream_t);

}  // namespace gdr
