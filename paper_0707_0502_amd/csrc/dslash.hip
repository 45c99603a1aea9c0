// Wilson-Dirac matrix-vector product (Sec. 4, Example 7's operator):
//   out = alpha * ((1 - sigma) in - kappa D in) [+ add]
//   D psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^H psi(x-mu)
// One thread per lattice site (both parities in one launch), even-odd SoA
// vectors so every component load is coalesced across a wavefront. Each
// hop is spin-projected to a 2-spinor, multiplied by the 3x3 link and
// reconstructed (the rank-2 projectors 1 -/+ g_mu of the chiral basis).
// The time-boundary factor is folded into the links at pack time. Blocks
// are remapped so that each XCD (blocks are dealt round-robin over the 8
// XCDs) works on one contiguous range of sites, keeping neighbour reuse in
// its own L2.
#include "kernels.h"

namespace gdr {

template <typename R>
struct Z {
    R x, y;
};
template <typename R>
__device__ __forceinline__ Z<R> zadd(Z<R> a, Z<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ Z<R> zsub(Z<R> a, Z<R> b) { return {a.x - b.x, a.y - b.y}; }
// a + s*i*b  (s = +1 or -1)
template <typename R>
__device__ __forceinline__ Z<R> zaddi(Z<R> a, Z<R> b, R s) { return {a.x - s * b.y, a.y + s * b.x}; }
template <typename R>
__device__ __forceinline__ Z<R> zaxs(Z<R> a, Z<R> b, R s) { return {a.x + s * b.x, a.y + s * b.y}; }
// s*i*b
template <typename R>
__device__ __forceinline__ Z<R> zi(Z<R> b, R s) { return {-s * b.y, s * b.x}; }
template <typename R>
__device__ __forceinline__ Z<R> zs(Z<R> b, R s) { return {s * b.x, s * b.y}; }

template <typename R>
__device__ __forceinline__ Z<R> ld(const double2* p) { double2 v = *p; return {(R)v.x, (R)v.y}; }
template <typename R>
__device__ __forceinline__ Z<R> ld(const float2* p) { float2 v = *p; return {(R)v.x, (R)v.y}; }
template <typename R>
__device__ __forceinline__ Z<R> ld(const __half2* p) {
    float2 v = __half22float2(*p);
    return {(R)v.x, (R)v.y};
}

// element at byte offset `off` (32-bit) from a uniform base: lets the
// compiler use scalar-base + 32-bit vector-offset addressing
template <typename X>
__device__ __forceinline__ const X* at(const X* base, unsigned off) {
    return (const X*)((const char*)base + off);
}

template <typename TS, typename TL, typename R>
struct DslashK {
    using C = typename CT<TS>::t;

    __device__ static void run(const C* __restrict__ in, int64_t in_stride, C* __restrict__ out,
                               int64_t out_stride, const C* __restrict__ add, int64_t add_stride,
                               const TL* __restrict__ links, const Geom& g, R kappa,
                               const DiagList& dl, const int* __restrict__ act) {
        const int v = blockIdx.y;
        if (act && !act[v]) return;
        const int nb = gridDim.x;
        const int b = blockIdx.x;
        const int lb = (nb % 8 == 0) ? ((b % 8) * (nb / 8) + b / 8) : b;
        // each block covers one parity, so every base pointer is uniform
        const int bpp = (g.vh + 255) / 256;
        const int p = lb >= bpp;
        const int s = (lb - p * bpp) * 256 + threadIdx.x;
        if (s >= g.vh) return;
        const int q = 1 - p;
        int c[4];
        {
            int r = s / g.hx;
            int xh = s - r * g.hx;
            c[1] = r % g.L[1];
            r /= g.L[1];
            c[2] = r % g.L[2];
            c[3] = r / g.L[2];
            c[0] = 2 * xh + ((p + c[1] + c[2] + c[3]) & 1);
        }
        const int64_t vh = g.vh;
        const C* inv = in + v * in_stride;
        const C* inq = inv + (int64_t)q * 12 * vh;

        Z<R> acc[4][3];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[sp][a] = {0, 0};

        // Spin projection of hop mu with sign sg (-1: forward with 1 - g_mu,
        // +1: backward with 1 + g_mu) in the chiral basis:
        //   h0 = psi0 + c0 psi_{p0},  h1 = psi1 + c1 psi_{p1},
        //   out rows 0,1 += U h0, U h1;  row p0 += conj(c0) U h0;  row p1 += conj(c1) U h1
        // with (p0, p1) = (3, 2) for mu = x, y and (2, 3) for mu = z, t, and
        //   mu=x: c0 = c1 = i sg;   mu=y: c0 = -sg, c1 = sg;
        //   mu=z: c0 = i sg, c1 = -i sg;   mu=t: c0 = c1 = sg.
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            const int L = g.L[mu];
            const int cm = mu == 0 ? c[0] : mu == 1 ? c[1] : mu == 2 ? c[2] : c[3];
            const int up = cm + 1 == L ? 0 : cm + 1;
            const int dn = cm == 0 ? L - 1 : cm - 1;
            const bool low = mu < 2;   // (p0, p1) = (3, 2)
#pragma unroll
            for (int dir = 0; dir < 2; ++dir) {
                const int cn = dir == 0 ? up : dn;
                const int x = mu == 0 ? cn : c[0];
                const int y = mu == 1 ? cn : c[1];
                const int zz = mu == 2 ? cn : c[2];
                const int tt = mu == 3 ? cn : c[3];
                const int sn = (x >> 1) + g.hx * (y + g.L[1] * (zz + g.L[2] * tt));
                const R sg = dir == 0 ? R(-1) : R(1);
                // c0, c1 as (re, im)
                R c0r, c0i, c1r, c1i;
                if (mu == 0) { c0r = 0; c0i = sg; c1r = 0; c1i = sg; }
                else if (mu == 1) { c0r = -sg; c0i = 0; c1r = sg; c1i = 0; }
                else if (mu == 2) { c0r = 0; c0i = sg; c1r = 0; c1i = -sg; }
                else { c0r = sg; c0i = 0; c1r = sg; c1i = 0; }
                Z<R> ps[4][3];
#pragma unroll
                for (int sp = 0; sp < 4; ++sp)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        ps[sp][a] = ld<R>(at(inq + (sp * 3 + a) * vh, (unsigned)sn * (unsigned)sizeof(C)));
                const int lp = dir == 0 ? p : q;
                const int ls = dir == 0 ? s : sn;
                const TL* lk = links + ((int64_t)(lp * 4 + mu) * 9) * vh;
                Z<R> u[3][3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int bb = 0; bb < 3; ++bb)
                        u[a][bb] = ld<R>(at(lk + (a * 3 + bb) * vh, (unsigned)ls * (unsigned)sizeof(TL)));
                Z<R> h0[3], h1[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const Z<R> q0 = low ? ps[3][a] : ps[2][a];
                    const Z<R> q1 = low ? ps[2][a] : ps[3][a];
                    h0[a] = {ps[0][a].x + c0r * q0.x - c0i * q0.y, ps[0][a].y + c0r * q0.y + c0i * q0.x};
                    h1[a] = {ps[1][a].x + c1r * q1.x - c1i * q1.y, ps[1][a].y + c1r * q1.y + c1i * q1.x};
                }
                Z<R> g0[3], g1[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    Z<R> s0 = {0, 0}, s1 = {0, 0};
#pragma unroll
                    for (int bb = 0; bb < 3; ++bb) {
                        // forward: U[a][bb]; backward: conj(U[bb][a])
                        const Z<R> m = dir == 0 ? u[a][bb] : Z<R>{u[bb][a].x, -u[bb][a].y};
                        s0.x += m.x * h0[bb].x - m.y * h0[bb].y;
                        s0.y += m.x * h0[bb].y + m.y * h0[bb].x;
                        s1.x += m.x * h1[bb].x - m.y * h1[bb].y;
                        s1.y += m.x * h1[bb].y + m.y * h1[bb].x;
                    }
                    g0[a] = s0;
                    g1[a] = s1;
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    acc[0][a] = zadd(acc[0][a], g0[a]);
                    acc[1][a] = zadd(acc[1][a], g1[a]);
                    // conj(c0) g0 and conj(c1) g1
                    const Z<R> e0 = {c0r * g0[a].x + c0i * g0[a].y, c0r * g0[a].y - c0i * g0[a].x};
                    const Z<R> e1 = {c1r * g1[a].x + c1i * g1[a].y, c1r * g1[a].y - c1i * g1[a].x};
                    acc[2][a] = zadd(acc[2][a], low ? e1 : e0);
                    acc[3][a] = zadd(acc[3][a], low ? e0 : e1);
                }
            }
        }
        const C* inp = inv + (int64_t)p * 12 * vh + s;
        C* o = out + v * out_stride + (int64_t)p * 12 * vh + s;
        const C* ad = add ? add + v * add_stride + (int64_t)p * 12 * vh + s : nullptr;
        const R dre = (R)dl.d[v].x, dim = (R)dl.d[v].y, al = (R)dl.alpha[v];
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int comp = sp * 3 + a;
                Z<R> xi = ld<R>(inp + comp * vh);
                R re = dre * xi.x - dim * xi.y - kappa * acc[sp][a].x;
                R im = dre * xi.y + dim * xi.x - kappa * acc[sp][a].y;
                re *= al;
                im *= al;
                if (ad) {
                    Z<R> av = ld<R>(ad + comp * vh);
                    re += av.x;
                    im += av.y;
                }
                C w;
                w.x = re;
                w.y = im;
                o[comp * vh] = w;
            }
    }
};

template <typename TS> struct DslashOcc { static constexpr int waves = 4; };
template <> struct DslashOcc<double> { static constexpr int waves = 2; };

template <typename TS, typename TL, typename R>
__global__ __launch_bounds__(256, DslashOcc<TS>::waves) void k_dslash(const typename CT<TS>::t* __restrict__ in,
                                                int64_t in_stride, typename CT<TS>::t* __restrict__ out,
                                                int64_t out_stride,
                                                const typename CT<TS>::t* __restrict__ add,
                                                int64_t add_stride, const TL* __restrict__ links,
                                                Geom g, R kappa, DiagList dl,
                                                const int* __restrict__ act) {
    DslashK<TS, TL, R>::run(in, in_stride, out, out_stride, add, add_stride, links, g, kappa, dl,
                            act);
}

template <typename TS>
void dslash(const typename CT<TS>::t* in, int64_t in_stride, typename CT<TS>::t* out,
            int64_t out_stride, const typename CT<TS>::t* add, int64_t add_stride,
            const void* links, int link_storage, const Geom& g, double kappa, const DiagList& dl,
            int nvec, hipStream_t st, const int* act) {
    dim3 grid(2 * ((g.vh + 255) / 256), nvec);
    if constexpr (std::is_same<TS, double>::value) {
        hipLaunchKernelGGL((k_dslash<double, double2, double>), grid, dim3(256), 0, st, in,
                           in_stride, out, out_stride, add, add_stride, (const double2*)links, g,
                           kappa, dl, act);
    } else {
        if (link_storage == 2) {
            hipLaunchKernelGGL((k_dslash<float, __half2, float>), grid, dim3(256), 0, st, in,
                               in_stride, out, out_stride, add, add_stride,
                               (const __half2*)links, g, (float)kappa, dl, act);
        } else {
            hipLaunchKernelGGL((k_dslash<float, float2, float>), grid, dim3(256), 0, st, in,
                               in_stride, out, out_stride, add, add_stride, (const float2*)links,
                               g, (float)kappa, dl, act);
        }
    }
}

template void dslash<double>(const double2*, int64_t, double2*, int64_t, const double2*, int64_t,
                             const void*, int, const Geom&, double, const DiagList&, int,
                             hipStream_t, const int*);
template void dslash<float>(const float2*, int64_t, float2*, int64_t, const float2*, int64_t,
                            const void*, int, const Geom&, double, const DiagList&, int,
                            hipStream_t, const int*);

}  // namespace gdr
