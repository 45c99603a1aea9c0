// Wilson-Dirac matrix-vector product (Sec. 4, Example 7's operator):
//   out = alpha * ((1 - sigma) in - kappa D in) [+ add]
//   D psi(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^H psi(x-mu)
// One thread per lattice site on the tile-blocked SoA layout (every
// component load is a contiguous run across a wavefront). A block covers
// 256 consecutive sites, i.e. whole tiles. Two kernels:
//  * k_dslash_halo (FP32 vectors, FP32 or FP16 links, 4^4 tiles): the block
//    stages its tile and the spin-projected halo of its eight faces in LDS,
//    so every hop reads its spinor from LDS;
//  * k_dslash (FP64, and FP32 on lattices with a tile extent of 2): the block
//    stages its own tile only; hops across a face read global memory.
// Each hop is spin-projected to a 2-spinor, multiplied by the 3x3 link and
// reconstructed (the rank-2 projectors 1 -/+ g_mu of the chiral basis). The
// time-boundary factor is folded into the links at pack time. Blocks are
// remapped so that each XCD (blocks are dealt round-robin over the 8 XCDs)
// works on one contiguous range of tiles, keeping the cross-face reuse in its
// own L2; a batched launch puts the blocks of one tile for all its vectors
// next to each other, so they share the tile's links through L2.
#include "kernels.h"
#include "tune.h"

#include <cstdio>
#include <stdexcept>
#include <type_traits>

namespace gdr {

template <typename R>
struct Z {
    R x, y;
};

// The operator's product is read by the next kernel from HBM in any case:
// non-temporal stores keep it from evicting the links and neighbour tiles
// that other blocks still read from L2.
typedef float f2o __attribute__((ext_vector_type(2)));
typedef double d2o __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st_nt(float2* p, float re, float im) {
    __builtin_nontemporal_store(f2o{re, im}, (f2o*)p);
}
__device__ __forceinline__ void st_nt(double2* p, double re, double im) {
    __builtin_nontemporal_store(d2o{re, im}, (d2o*)p);
}
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

// c q for c = CR + i CI with CR, CI in {-1, 0, 1} (one of them zero): a
// swap and sign changes, no multiplications
template <int CR, int CI, typename R>
__device__ __forceinline__ Z<R> mulc(Z<R> q) {
    if constexpr (CR == 0) {
        if constexpr (CI == 1) return {-q.y, q.x};
        else return {q.y, -q.x};
    } else {
        if constexpr (CR == 1) return q;
        else return {-q.x, -q.y};
    }
}

// One hop with its direction fixed at compile time. Spin projection of hop
// MU with sign sg (-1: forward with 1 - g_mu, +1: backward with 1 + g_mu) in
// the chiral basis:
//   h0 = psi0 + c0 psi_{p0},  h1 = psi1 + c1 psi_{p1},
//   out rows 0,1 += U h0, U h1;  row p0 += conj(c0) U h0;  row p1 += conj(c1) U h1
// with (p0, p1) = (3, 2) for mu = x, y and (2, 3) for mu = z, t, and
//   mu=x: c0 = c1 = i sg;   mu=y: c0 = -sg, c1 = sg;
//   mu=z: c0 = i sg, c1 = -i sg;   mu=t: c0 = c1 = sg.
// Forward hops multiply by U_mu(x), backward hops by U_mu(x - mu)^H.
template <int MU, int DIR>
struct HopC {
    static constexpr int sg = DIR == 0 ? -1 : 1;
    static constexpr int c0r = MU == 1 ? -sg : MU == 3 ? sg : 0;
    static constexpr int c0i = MU == 0 || MU == 2 ? sg : 0;
    static constexpr int c1r = MU == 1 || MU == 3 ? sg : 0;
    static constexpr int c1i = MU == 0 ? sg : MU == 2 ? -sg : 0;
    static constexpr bool low = MU < 2;   // (p0, p1) = (3, 2)
};

// spin projection of a full spinor for hop (MU, DIR): the half spinor (h0, h1)
template <int MU, int DIR, typename R>
__device__ __forceinline__ void proj(const Z<R> (&ps)[4][3], Z<R> (&h0)[3], Z<R> (&h1)[3]) {
    using H = HopC<MU, DIR>;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        h0[a] = zadd(ps[0][a], mulc<H::c0r, H::c0i>(H::low ? ps[3][a] : ps[2][a]));
        h1[a] = zadd(ps[1][a], mulc<H::c1r, H::c1i>(H::low ? ps[2][a] : ps[3][a]));
    }
}

// link times half spinor, reconstructed into the four spin rows of acc
template <int MU, int DIR, typename R>
__device__ __forceinline__ void mulrec(Z<R> (&acc)[4][3], const Z<R> (&h0)[3], const Z<R> (&h1)[3],
                                       const Z<R> (&u)[3][3]) {
    using H = HopC<MU, DIR>;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        // (U h)_a; the first term starts the sum (an added zero would not be
        // folded away under IEEE rules)
        Z<R> s0, s1;
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            const Z<R> m = DIR == 0 ? u[a][bb] : Z<R>{u[bb][a].x, -u[bb][a].y};
            const Z<R> t0 = {m.x * h0[bb].x - m.y * h0[bb].y, m.x * h0[bb].y + m.y * h0[bb].x};
            const Z<R> t1 = {m.x * h1[bb].x - m.y * h1[bb].y, m.x * h1[bb].y + m.y * h1[bb].x};
            s0 = bb == 0 ? t0 : zadd(s0, t0);
            s1 = bb == 0 ? t1 : zadd(s1, t1);
        }
        acc[0][a] = zadd(acc[0][a], s0);
        acc[1][a] = zadd(acc[1][a], s1);
        const Z<R> e0 = mulc<H::c0r, -H::c0i>(s0);   // conj(c0) U h0
        const Z<R> e1 = mulc<H::c1r, -H::c1i>(s1);
        acc[2][a] = zadd(acc[2][a], H::low ? e1 : e0);
        acc[3][a] = zadd(acc[3][a], H::low ? e0 : e1);
    }
}

// An empty asm that claims to change x: the compiler must have x ready at
// this point and cannot compute anything derived from the new value earlier.
// Used to keep the eight hops in sequence (otherwise the straight-line code
// is reordered so that all loads come first and the registers spill).
template <typename X>
__device__ __forceinline__ void pin(X& x) {
    asm volatile("" : "+v"(x));
}

template <typename TS, typename TL, typename R>
struct DslashK {
    using C = typename CT<TS>::t;

    __device__ static void run(const C* __restrict__ in, int64_t in_stride, C* __restrict__ out,
                               int64_t out_stride, const C* __restrict__ add, int64_t add_stride,
                               const TL* __restrict__ links, const Geom& g, R kappa,
                               const DiagList& dl, const int* __restrict__ act, int nvec) {
        __shared__ C sp[12 * 256];
        // blocks of one tile range for all nvec vectors are consecutive, so a
        // batched launch reads each link from HBM once and from L2 after that
        const int nb = gridDim.x;
        const int b = blockIdx.x;
        const int lbv = (nb % 8 == 0) ? ((b % 8) * (nb / 8) + b / 8) : b;
        const int v = lbv % nvec;
        const int lb = lbv / nvec;
        if (act && !act[v]) return;   // inactive member: uniform over the block, nothing loaded
        const int local = threadIdx.x;
        const int site0 = lb * 256 + local;
        const int vol = g.vol;
        const bool valid = site0 < vol;   // blocks hold whole tiles: a tile is all valid or all not
        const int64_t V = vol;
        const C* inv = in + v * in_stride;
        // all twelve loads in flight at once: sites past the volume read
        // site 0 (in bounds) and stage zeros
        const int ss = valid ? site0 : 0;
        C st[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) st[c] = inv[c * V + ss];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            if (!valid) {
                st[c].x = 0;
                st[c].y = 0;
            }
            sp[c * 256 + local] = st[c];
        }
        __syncthreads();
        if (!valid) return;
        const int ltv = g.ltv;
        const int T0 = site0 >> ltv;
        const int w0 = site0 & ((1 << ltv) - 1);
        const int slot = local & ~((1 << ltv) - 1);   // first LDS slot of this tile
        int tc[4];
        {
            int r = T0;
            tc[0] = r % g.nt[0];
            r /= g.nt[0];
            tc[1] = r % g.nt[1];
            r /= g.nt[1];
            tc[2] = r % g.nt[2];
            tc[3] = r / g.nt[2];
        }
        const int tst[4] = {1, g.nt[0], g.nt[0] * g.nt[1], g.nt[0] * g.nt[1] * g.nt[2]};

        Z<R> acc[4][3];
#pragma unroll
        for (int sp_ = 0; sp_ < 4; ++sp_)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[sp_][a] = {0, 0};

        // the eight hops, each with its projection constants fixed at
        // compile time; a hop inside the tile reads LDS, across a face global
        // memory (the neighbouring tile, periodic wrap)
        auto hop = [&](auto muc, auto dirc) {
            constexpr int mu = decltype(muc)::value;
            constexpr int dir = decltype(dirc)::value;
            int w = w0, T = T0, site = site0;
            pin(w);
            pin(T);
            pin(site);
            const int offm = g.off[mu];
            const int bm = 1 << g.lb[mu];
            const int cm = (w >> offm) & (bm - 1);
            const int ntm = g.nt[mu];
            const int tcm = tc[mu];
            const int stm = tst[mu];
            const bool inside = dir == 0 ? cm < bm - 1 : cm > 0;
            int wn, Tn;
            if (dir == 0) {
                wn = inside ? w + (1 << offm) : w - ((bm - 1) << offm);
                Tn = inside ? T : (tcm == ntm - 1 ? T - (ntm - 1) * stm : T + stm);
            } else {
                wn = inside ? w - (1 << offm) : w + ((bm - 1) << offm);
                Tn = inside ? T : (tcm == 0 ? T + (ntm - 1) * stm : T - stm);
            }
            const int sn = (Tn << ltv) | wn;
            Z<R> ps[4][3];
            if (inside) {
                const int li = slot + wn;
#pragma unroll
                for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                    for (int a = 0; a < 3; ++a) ps[s_][a] = ld<R>(&sp[(s_ * 3 + a) * 256 + li]);
            } else {
#pragma unroll
                for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                    for (int a = 0; a < 3; ++a)
                        ps[s_][a] = ld<R>(at(inv + (s_ * 3 + a) * V, (unsigned)sn * (unsigned)sizeof(C)));
            }
            const TL* lk = links + (int64_t)mu * 9 * V;
            const int ls = dir == 0 ? site : sn;
            Z<R> u[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
                    u[a][bb] = ld<R>(at(lk + (a * 3 + bb) * V, (unsigned)ls * (unsigned)sizeof(TL)));
            Z<R> h0[3], h1[3];
            proj<mu, dir>(ps, h0, h1);
            mulrec<mu, dir>(acc, h0, h1, u);
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    pin(acc[s_][a].x);
                    pin(acc[s_][a].y);
                }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        hop(I0{}, I0{});
        hop(I0{}, I1{});
        hop(I1{}, I0{});
        hop(I1{}, I1{});
        hop(I2{}, I0{});
        hop(I2{}, I1{});
        hop(I3{}, I0{});
        hop(I3{}, I1{});

        int site = site0, lsl = local;
        pin(site);
        pin(lsl);
        C* o = out + v * out_stride + site;
        const C* ad = add ? add + v * add_stride + site : nullptr;
        const R dre = (R)dl.d[v].x, dim = (R)dl.d[v].y, al = (R)dl.alpha[v];
        auto fin = [&](auto with_add) {
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int comp = s_ * 3 + a;
                    Z<R> xi = ld<R>(&sp[comp * 256 + lsl]);
                    R re = dre * xi.x - dim * xi.y - kappa * acc[s_][a].x;
                    R im = dre * xi.y + dim * xi.x - kappa * acc[s_][a].y;
                    re *= al;
                    im *= al;
                    if constexpr (decltype(with_add)::value) {
                        Z<R> av = ld<R>(ad + comp * V);
                        re += av.x;
                        im += av.y;
                    }
                    st_nt(&o[comp * V], re, im);
                }
        };
        if (ad) fin(std::true_type{});
        else fin(std::false_type{});
    }
};

// FP32 operator for lattices cut into 4^4 tiles (every extent a multiple of
// 4): a block of 256 threads is one tile. Before any hop it stages, with all
// loads in flight together, its own tile and the spin-projected halo: for
// each of the eight faces the 64 neighbouring sites across that face,
// projected with that hop's (1 -/+ g_mu) to half spinors (6 complex). Every
// hop then reads spinors from LDS only (inside the tile the full neighbour,
// projected in the hop; across a face the staged half spinor), so no hop
// waits on a scattered global read; the links still come from global
// memory. LDS 48 KB per block (3 blocks per CU).
template <typename TL>
struct DslashHaloK {
    using C = float2;
    using R = float;

    __device__ static void run(const C* __restrict__ in, int64_t in_stride, C* __restrict__ out,
                               int64_t out_stride, const C* __restrict__ add, int64_t add_stride,
                               const TL* __restrict__ links, const Geom& g, R kappa,
                               const DiagList& dl, const int* __restrict__ act, int nvec) {
        __shared__ C sp[12 * 256];        // own tile, [component][site]
        __shared__ C hl[8 * 6 * 64];      // halo, [face = 2 mu + dir][half-spinor component][face site]
        const int nb = gridDim.x;
        const int b = blockIdx.x;
        const int lbv = (nb % 8 == 0) ? ((b % 8) * (nb / 8) + b / 8) : b;
        const int v = lbv % nvec;
        const int T = lbv / nvec;   // tile
        if (act && !act[v]) return;   // inactive member: uniform over the block, nothing loaded
        const int local = threadIdx.x;
        const int site0 = (T << 8) | local;
        const int64_t V = g.vol;
        const C* inv = in + v * in_stride;
        int tc[4];
        {
            int r = T;
            tc[0] = r % g.nt[0];
            r /= g.nt[0];
            tc[1] = r % g.nt[1];
            r /= g.nt[1];
            tc[2] = r % g.nt[2];
            tc[3] = r / g.nt[2];
        }
        const int tst[4] = {1, g.nt[0], g.nt[0] * g.nt[1], g.nt[0] * g.nt[1] * g.nt[2]};
        // neighbouring tile along mu (forward or backward, periodic)
        auto ntile = [&](int mu, int dir) {
            const int ntm = mu == 0 ? g.nt[0] : mu == 1 ? g.nt[1] : mu == 2 ? g.nt[2] : g.nt[3];
            const int tcm = mu == 0 ? tc[0] : mu == 1 ? tc[1] : mu == 2 ? tc[2] : tc[3];
            const int stm = mu == 0 ? tst[0] : mu == 1 ? tst[1] : mu == 2 ? tst[2] : tst[3];
            return dir == 0 ? (tcm == ntm - 1 ? T - (ntm - 1) * stm : T + stm)
                            : (tcm == 0 ? T + (ntm - 1) * stm : T - stm);
        };

        // ---- staging: own site, and halo entries e = local and local + 256
        // (face f = e / 64 is uniform over a wavefront, j = e % 64 the face site)
        C st[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) st[c] = inv[c * V + site0];
        C hs[2][12];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = local + 256 * h;
            const int f = e >> 6, j = e & 63;
            const int mu = f >> 1, dir = f & 1;
            const int sh = 2 * mu;
            // the neighbour across face (mu, dir): coordinate mu is 0 in the
            // next tile (forward) or 3 in the previous one (backward), the
            // other three are those of face site j
            const int cn = dir == 0 ? 0 : 3;
            const int wn = (j & ((1 << sh) - 1)) | (cn << sh) | ((j >> sh) << (sh + 2));
            const int sn = (ntile(mu, dir) << 8) | wn;
#pragma unroll
            for (int c = 0; c < 12; ++c) hs[h][c] = *at(inv + c * V, (unsigned)sn * (unsigned)sizeof(C));
        }
#pragma unroll
        for (int c = 0; c < 12; ++c) sp[c * 256 + local] = st[c];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = local + 256 * h;
            const int f = e >> 6, j = e & 63;
            Z<R> ps[4][3], h0[3], h1[3];
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int a = 0; a < 3; ++a) ps[s_][a] = {hs[h][s_ * 3 + a].x, hs[h][s_ * 3 + a].y};
            switch (f) {
                case 0: proj<0, 0>(ps, h0, h1); break;
                case 1: proj<0, 1>(ps, h0, h1); break;
                case 2: proj<1, 0>(ps, h0, h1); break;
                case 3: proj<1, 1>(ps, h0, h1); break;
                case 4: proj<2, 0>(ps, h0, h1); break;
                case 5: proj<2, 1>(ps, h0, h1); break;
                case 6: proj<3, 0>(ps, h0, h1); break;
                default: proj<3, 1>(ps, h0, h1); break;
            }
            C* hp = hl + f * 6 * 64 + j;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                hp[a * 64] = make_float2(h0[a].x, h0[a].y);
                hp[(3 + a) * 64] = make_float2(h1[a].x, h1[a].y);
            }
        }
        __syncthreads();

        Z<R> acc[4][3];
#pragma unroll
        for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[s_][a] = {0, 0};
        auto hop = [&](auto muc, auto dirc) {
            constexpr int mu = decltype(muc)::value;
            constexpr int dir = decltype(dirc)::value;
            constexpr int sh = 2 * mu;
            int w = local, site = site0;
            pin(w);
            pin(site);
            const int cm = (w >> sh) & 3;
            const bool inside = dir == 0 ? cm < 3 : cm > 0;
            const int wn = dir == 0 ? (inside ? w + (1 << sh) : w - (3 << sh))
                                    : (inside ? w - (1 << sh) : w + (3 << sh));
            Z<R> h0[3], h1[3];
            if (inside) {
                Z<R> ps[4][3];
#pragma unroll
                for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                    for (int a = 0; a < 3; ++a) ps[s_][a] = ld<R>(&sp[(s_ * 3 + a) * 256 + wn]);
                proj<mu, dir>(ps, h0, h1);
            } else {
                const int j = (w & ((1 << sh) - 1)) | ((w >> (sh + 2)) << sh);
                const C* hp = hl + (2 * mu + dir) * 6 * 64 + j;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    h0[a] = ld<R>(&hp[a * 64]);
                    h1[a] = ld<R>(&hp[(3 + a) * 64]);
                }
            }
            // forward: U_mu(x) at this site; backward: U_mu(x - mu) at the
            // neighbour, in the previous tile for face sites
            int ls = site;
            if (dir == 1) ls = ((inside ? T : ntile(mu, 1)) << 8) | wn;
            const TL* lk = links + (int64_t)mu * 9 * V;
            Z<R> u[3][3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int bb = 0; bb < 3; ++bb)
                    u[a][bb] = ld<R>(at(lk + (a * 3 + bb) * V, (unsigned)ls * (unsigned)sizeof(TL)));
            mulrec<mu, dir>(acc, h0, h1, u);
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    pin(acc[s_][a].x);
                    pin(acc[s_][a].y);
                }
        };
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        using I3 = std::integral_constant<int, 3>;
        hop(I0{}, I0{});
        hop(I0{}, I1{});
        hop(I1{}, I0{});
        hop(I1{}, I1{});
        hop(I2{}, I0{});
        hop(I2{}, I1{});
        hop(I3{}, I0{});
        hop(I3{}, I1{});

        int site = site0, lsl = local;
        pin(site);
        pin(lsl);
        C* o = out + v * out_stride + site;
        const C* ad = add ? add + v * add_stride + site : nullptr;
        const R dre = (R)dl.d[v].x, dim = (R)dl.d[v].y, al = (R)dl.alpha[v];
        auto fin = [&](auto with_add) {
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int comp = s_ * 3 + a;
                    Z<R> xi = ld<R>(&sp[comp * 256 + lsl]);
                    R re = al * (dre * xi.x - dim * xi.y - kappa * acc[s_][a].x);
                    R im = al * (dre * xi.y + dim * xi.x - kappa * acc[s_][a].y);
                    if constexpr (decltype(with_add)::value) {
                        Z<R> av = ld<R>(ad + comp * V);
                        re += av.x;
                        im += av.y;
                    }
                    st_nt(&o[comp * V], re, im);
                }
        };
        if (ad) fin(std::true_type{});
        else fin(std::false_type{});
    }
};

// ---------------------------------------------------------------------------
// FP32 operator on special unitary links stored as their first two rows
// (LINK_R12: 12 reals instead of 18 per link, a third less link traffic);
// the third row is rebuilt as conj(row0 x row1), exact for det U = 1, and the
// boundary factor bc[mu] = -1 is applied here on the last slice (the stored
// links carry none, since -U is not special unitary). 4^4 tiles only.

// link of one hop: rows 0 and 1 at site ls (FP32 or FP16 entries), row 2
// rebuilt in FP32
template <typename LT>
__device__ __forceinline__ void ld_r12(const LT* __restrict__ lk, int64_t V, int ls,
                                       Z<float> (&u)[3][3]) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
            u[a][bb] = ld<float>(at(lk + (a * 3 + bb) * V, (unsigned)ls * (unsigned)sizeof(LT)));
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
        const int b1 = (bb + 1) % 3, b2 = (bb + 2) % 3;
        // conj(u0[b1] u1[b2] - u0[b2] u1[b1])
        float re = u[0][b1].x * u[1][b2].x;
        float im = u[0][b1].x * u[1][b2].y;
        re = __builtin_fmaf(-u[0][b1].y, u[1][b2].y, re);
        im = __builtin_fmaf(u[0][b1].y, u[1][b2].x, im);
        re = __builtin_fmaf(-u[0][b2].x, u[1][b1].x, re);
        im = __builtin_fmaf(-u[0][b2].x, u[1][b1].y, im);
        re = __builtin_fmaf(u[0][b2].y, u[1][b1].y, re);
        im = __builtin_fmaf(-u[0][b2].y, u[1][b1].x, im);
        u[2][bb] = {re, -im};
    }
}

// mulrec with explicit FMA chains and a sign sg = +-1 on the whole hop
template <int MU, int DIR>
__device__ __forceinline__ void mulrec_sg(Z<float> (&acc)[4][3], const Z<float> (&h0)[3],
                                          const Z<float> (&h1)[3], const Z<float> (&u)[3][3],
                                          float sg) {
    using H = HopC<MU, DIR>;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float s0x, s0y, s1x, s1y;
#pragma unroll
        for (int bb = 0; bb < 3; ++bb) {
            // m = u[a][bb] (forward) or conj(u[bb][a]) (backward)
            const float mx = DIR == 0 ? u[a][bb].x : u[bb][a].x;
            const float my = DIR == 0 ? u[a][bb].y : -u[bb][a].y;
            if (bb == 0) {
                s0x = mx * h0[0].x;
                s0y = mx * h0[0].y;
                s1x = mx * h1[0].x;
                s1y = mx * h1[0].y;
            } else {
                s0x = __builtin_fmaf(mx, h0[bb].x, s0x);
                s0y = __builtin_fmaf(mx, h0[bb].y, s0y);
                s1x = __builtin_fmaf(mx, h1[bb].x, s1x);
                s1y = __builtin_fmaf(mx, h1[bb].y, s1y);
            }
            s0x = __builtin_fmaf(-my, h0[bb].y, s0x);
            s0y = __builtin_fmaf(my, h0[bb].x, s0y);
            s1x = __builtin_fmaf(-my, h1[bb].y, s1x);
            s1y = __builtin_fmaf(my, h1[bb].x, s1y);
        }
        const Z<float> s0{s0x, s0y}, s1{s1x, s1y};
        const Z<float> e0 = mulc<H::c0r, -H::c0i>(s0);   // conj(c0) U h0
        const Z<float> e1 = mulc<H::c1r, -H::c1i>(s1);
        const Z<float> r2 = H::low ? e1 : e0, r3 = H::low ? e0 : e1;
        acc[0][a] = {__builtin_fmaf(sg, s0.x, acc[0][a].x), __builtin_fmaf(sg, s0.y, acc[0][a].y)};
        acc[1][a] = {__builtin_fmaf(sg, s1.x, acc[1][a].x), __builtin_fmaf(sg, s1.y, acc[1][a].y)};
        acc[2][a] = {__builtin_fmaf(sg, r2.x, acc[2][a].x), __builtin_fmaf(sg, r2.y, acc[2][a].y)};
        acc[3][a] = {__builtin_fmaf(sg, r3.x, acc[3][a].x), __builtin_fmaf(sg, r3.y, acc[3][a].y)};
    }
}

// Geometry of one 4^4 tile T: tile coordinates and the neighbouring tile
// across each face (periodic wrap). Scalar fields only: a per-direction
// array indexed by a run-time direction would be placed in scratch memory.
struct TileGeo {
    int T;
    int tc0, tc1, tc2, tc3;   // tile coordinates
    int nt0, nt1, nt2, nt3;   // tiles per direction
    int s1, s2, s3;           // tile index strides of y, z, t
    __device__ __forceinline__ TileGeo(const Geom& gg, int T_) : T(T_) {
        nt0 = gg.nt[0];
        nt1 = gg.nt[1];
        nt2 = gg.nt[2];
        nt3 = gg.nt[3];
        int r = T;
        tc0 = r % nt0;
        r /= nt0;
        tc1 = r % nt1;
        r /= nt1;
        tc2 = r % nt2;
        tc3 = r / nt2;
        s1 = nt0;
        s2 = nt0 * nt1;
        s3 = s2 * nt2;
    }
    template <int MU>
    __device__ __forceinline__ int tcoord() const {
        return MU == 0 ? tc0 : MU == 1 ? tc1 : MU == 2 ? tc2 : tc3;
    }
    template <int MU>
    __device__ __forceinline__ int ntiles() const {
        return MU == 0 ? nt0 : MU == 1 ? nt1 : MU == 2 ? nt2 : nt3;
    }
    template <int MU>
    __device__ __forceinline__ int nbr(int dir) const {
        const int ntm = ntiles<MU>(), tcm = tcoord<MU>();
        const int stm = MU == 0 ? 1 : MU == 1 ? s1 : MU == 2 ? s2 : s3;
        return dir == 0 ? (tcm == ntm - 1 ? T - (ntm - 1) * stm : T + stm)
                        : (tcm == 0 ? T + (ntm - 1) * stm : T - stm);
    }
    // run-time direction (uniform over a wavefront where it is used)
    __device__ __forceinline__ int nbr(int mu, int dir) const {
        if (mu == 0) return nbr<0>(dir);
        if (mu == 1) return nbr<1>(dir);
        if (mu == 2) return nbr<2>(dir);
        return nbr<3>(dir);
    }
};

// Tile of sequence position q (per XCD, after the block remap) in tile order
// `order`: 0 lexicographic (x fastest); 1 whole xy planes of tiles, then
// 2 x 2 blocks of (z, t) tile coordinates (needs nt2 and nt3 even), so that
// z and t neighbours come closer in the sequence
__device__ __forceinline__ int tile_of(const Geom& g, int q, int order) {
    if (order == 0) return q;
    const int nxy = g.nt[0] * g.nt[1];
    const int txy = q % nxy;
    int r = q / nxy;
    const int zl = r & 1, tl = (r >> 1) & 1;
    r >>= 2;
    const int zb = r % (g.nt[2] >> 1), tb = r / (g.nt[2] >> 1);
    return txy + nxy * ((2 * zb + zl) + g.nt[2] * (2 * tb + tl));
}

// storage index of face entry e (0..511) of tile geometry tg: face f = e / 64
// (2 mu + dir), site j = e % 64 across that face in the neighbouring tile
__device__ __forceinline__ int halo_source(const TileGeo tg, int e) {
    const int f = __builtin_amdgcn_readfirstlane(e >> 6), j = e & 63;   // f: one face per wavefront
    const int mu = f >> 1, dir = f & 1;
    const int sh = 2 * mu;
    const int cn = dir == 0 ? 0 : 3;
    const int wn = (j & ((1 << sh) - 1)) | (cn << sh) | ((j >> sh) << (sh + 2));
    return (tg.nbr(mu, dir) << 8) | wn;
}

// Load this thread's own site and its two halo entries of vector `inv` and
// stage them into LDS: the tile in sp[component][site], the spin-projected
// halo in hl[face][half-spinor component][face site]. SPLIT: in two rounds of
// loads (own site and first halo entry, then the second halo entry) instead
// of all 36 at once, for kernels that also hold the links in registers.
template <bool SPLIT>
__device__ __forceinline__ void stage_r12(const float2* __restrict__ inv, int64_t V, int site0,
                                          int local, const int (&hsrc)[2], float2* sp, float2* hl) {
    float2 st[12], hs[2][12];
#pragma unroll
    for (int c = 0; c < 12; ++c) st[c] = inv[c * V + site0];
#pragma unroll
    for (int h = 0; h < (SPLIT ? 1 : 2); ++h)
#pragma unroll
        for (int c = 0; c < 12; ++c) hs[h][c] = *at(inv + c * V, (unsigned)hsrc[h] * 8u);
#pragma unroll
    for (int c = 0; c < 12; ++c) sp[c * 256 + local] = st[c];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (SPLIT && h == 1) {
#pragma unroll
            for (int c = 0; c < 12; ++c) hs[1][c] = *at(inv + c * V, (unsigned)hsrc[1] * 8u);
        }
        const int e = local + 256 * h;
        const int f = e >> 6, j = e & 63;
        Z<float> ps[4][3], h0[3], h1[3];
#pragma unroll
        for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
            for (int a = 0; a < 3; ++a) ps[s_][a] = {hs[h][s_ * 3 + a].x, hs[h][s_ * 3 + a].y};
        switch (f) {
            case 0: proj<0, 0>(ps, h0, h1); break;
            case 1: proj<0, 1>(ps, h0, h1); break;
            case 2: proj<1, 0>(ps, h0, h1); break;
            case 3: proj<1, 1>(ps, h0, h1); break;
            case 4: proj<2, 0>(ps, h0, h1); break;
            case 5: proj<2, 1>(ps, h0, h1); break;
            case 6: proj<3, 0>(ps, h0, h1); break;
            default: proj<3, 1>(ps, h0, h1); break;
        }
        float2* hp = hl + f * 6 * 64 + j;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            hp[a * 64] = make_float2(h0[a].x, h0[a].y);
            hp[(3 + a) * 64] = make_float2(h1[a].x, h1[a].y);
        }
    }
}

// The spin-projected half spinor of hop (MU, DIR) at in-tile site w: from the
// staged tile (projected here) or the staged halo.
template <int MU, int DIR>
__device__ __forceinline__ void hop_input(const float2* sp, const float2* hl, int w, Z<float> (&h0)[3],
                                          Z<float> (&h1)[3]) {
    constexpr int sh = 2 * MU;
    const int cm = (w >> sh) & 3;
    const bool inside = DIR == 0 ? cm < 3 : cm > 0;
    if (inside) {
        const int wn = DIR == 0 ? w + (1 << sh) : w - (1 << sh);
        Z<float> ps[4][3];
#pragma unroll
        for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
            for (int a = 0; a < 3; ++a) ps[s_][a] = ld<float>(&sp[(s_ * 3 + a) * 256 + wn]);
        proj<MU, DIR>(ps, h0, h1);
    } else {
        const int j = (w & ((1 << sh) - 1)) | ((w >> (sh + 2)) << sh);
        const float2* hp = hl + (2 * MU + DIR) * 6 * 64 + j;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            h0[a] = ld<float>(&hp[a * 64]);
            h1[a] = ld<float>(&hp[(3 + a) * 64]);
        }
    }
}

// link site and boundary sign of hop (MU, DIR) at in-tile site w of tile tg
template <int MU, int DIR>
__device__ __forceinline__ void hop_link(const TileGeo tg, int w, int anti, int& ls, float& sg) {
    constexpr int sh = 2 * MU;
    const int cm = (w >> sh) & 3;
    const int ntm = tg.ntiles<MU>();
    if (DIR == 0) {
        ls = (tg.T << 8) | w;   // U_mu(x)
        sg = ((anti >> MU) & 1) && cm == 3 && tg.tcoord<MU>() == ntm - 1 ? -1.f : 1.f;
    } else {
        const bool inside = cm > 0;
        const int wn = inside ? w - (1 << sh) : w + (3 << sh);
        ls = ((inside ? tg.T : tg.nbr<MU>(1)) << 8) | wn;   // U_mu(x - mu)
        sg = ((anti >> MU) & 1) && cm == 0 && tg.tcoord<MU>() == 0 ? -1.f : 1.f;
    }
}

// out = alpha ((1 - sigma) in - kappa acc) [+ add], non-temporal stores
__device__ __forceinline__ void finish_r12(const Z<float> (&acc)[4][3], const float2* sp, int local,
                                           float2* o, const float2* ad, int64_t V, float dre, float dim,
                                           float al, float kappa) {
#pragma unroll
    for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int comp = s_ * 3 + a;
            const Z<float> xi = ld<float>(&sp[comp * 256 + local]);
            float re = al * (dre * xi.x - dim * xi.y - kappa * acc[s_][a].x);
            float im = al * (dre * xi.y + dim * xi.x - kappa * acc[s_][a].y);
            if (ad) {
                const Z<float> av = ld<float>(ad + comp * V);
                re += av.x;
                im += av.y;
            }
            st_nt(&o[comp * V], re, im);
        }
}

// One tile of one vector with two-row links (LT = float2: LINK_R12, __half2:
// LINK_R12H): stage the tile and its spin-projected halo, apply the eight
// hops, write alpha ((1 - sigma) in - kappa D in) [+ add]. in, out and add
// point at the vector's start; sp and hl are the block's LDS staging areas.
template <typename LT>
__device__ __forceinline__ void r12_tile(const float2* __restrict__ in, float2* __restrict__ out,
                                         const float2* __restrict__ add, const LT* __restrict__ links,
                                         const TileGeo& tg, int64_t V, float kappa, double2 d,
                                         double alpha, int anti, float2* sp, float2* hl) {
    const int local = threadIdx.x;
    const int site0 = (tg.T << 8) | local;
    const int hsrc[2] = {halo_source(tg, local), halo_source(tg, local + 256)};
    stage_r12<false>(in, V, site0, local, hsrc, sp, hl);
    __syncthreads();
    Z<float> acc[4][3];
#pragma unroll
    for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[s_][a] = {0, 0};
    auto hop = [&](auto muc, auto dirc) {
        constexpr int mu = decltype(muc)::value;
        constexpr int dir = decltype(dirc)::value;
        int w = local;
        pin(w);
        Z<float> h0[3], h1[3];
        hop_input<mu, dir>(sp, hl, w, h0, h1);
        int ls;
        float sg;
        hop_link<mu, dir>(tg, w, anti, ls, sg);
        Z<float> u[3][3];
        ld_r12(links + (int64_t)mu * 6 * V, V, ls, u);
        mulrec_sg<mu, dir>(acc, h0, h1, u, sg);
#pragma unroll
        for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                pin(acc[s_][a].x);
                pin(acc[s_][a].y);
            }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    hop(I0{}, I0{});
    hop(I0{}, I1{});
    hop(I1{}, I0{});
    hop(I1{}, I1{});
    hop(I2{}, I0{});
    hop(I2{}, I1{});
    hop(I3{}, I0{});
    hop(I3{}, I1{});
    finish_r12(acc, sp, local, out + site0, add ? add + site0 : nullptr, V, (float)d.x, (float)d.y,
               (float)alpha, kappa);
}

// One block per (tile, vector) with two-row links.
template <typename LT>
__global__ __launch_bounds__(256, 3) void k_dslash_r12(const float2* __restrict__ in, int64_t in_stride,
                                                      float2* __restrict__ out, int64_t out_stride,
                                                      const float2* __restrict__ add, int64_t add_stride,
                                                      const LT* __restrict__ links, Geom g, float kappa,
                                                      DiagList dl, const int* __restrict__ act, int nvec,
                                                      int anti, int order) {
    __shared__ float2 sp[12 * 256];
    __shared__ float2 hl[8 * 6 * 64];
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int lbv = (nb % 8 == 0) ? ((b % 8) * (nb / 8) + b / 8) : b;
    const int v = lbv % nvec;
    if (act && !act[v]) return;   // inactive member: uniform over the block, nothing loaded
    const TileGeo tg(g, tile_of(g, lbv / nvec, order));
    r12_tile<LT>(in + v * in_stride, out + v * out_stride, add ? add + v * add_stride : nullptr,
                 links, tg, g.vol, kappa, dl.d[v], dl.alpha[v], anti, sp, hl);
}

// Persistent work list over the vectors of several lattices (member v on
// lattice L.g[v], its vector at in + v * in_stride): items are the (member,
// tile) pairs in member order, and a grid of at most the resident blocks
// takes them in turn (item = block, block + grid, ...), so one launch serves
// every lattice however uneven their sizes. Inactive members cost one flag
// read per item.
template <typename LT>
__global__ __launch_bounds__(256, 3) void k_dslash_r12_list(const float2* __restrict__ in,
                                                           int64_t in_stride, float2* __restrict__ out,
                                                           int64_t out_stride, LatList L, DiagList dl,
                                                           const int* __restrict__ act) {
    __shared__ float2 sp[12 * 256];
    __shared__ float2 hl[8 * 6 * 64];
    const int total = L.tile0[L.nm];
    for (int item = blockIdx.x; item < total; item += gridDim.x) {
        int v = 0;
        while (v + 1 < L.nm && item >= L.tile0[v + 1]) ++v;
        if (act && !act[v]) continue;   // uniform over the block
        const Geom& g = L.g[v];
        const TileGeo tg(g, item - L.tile0[v]);
        r12_tile<LT>(in + v * in_stride, out + v * out_stride, nullptr, (const LT*)L.links[v], tg,
                     g.vol, L.kappa[v], dl.d[v], dl.alpha[v], L.anti[v], sp, hl);
        __syncthreads();   // the staging areas are reused by the next item
    }
}

// Several vectors per launch: one block per tile loops over the vectors. The
// links of the tile's eight hops (each link once, third row rebuilt once,
// boundary sign folded in) stay in registers for every vector; each vector
// is staged and applied as in k_dslash_r12 (no added vector: launches with
// one go to k_dslash_r12). Inactive members are skipped.
template <typename LT>
__global__ __launch_bounds__(256, 2) void k_dslash_r12v(const float2* __restrict__ in, int64_t in_stride,
                                                       float2* __restrict__ out, int64_t out_stride,
                                                       const LT* __restrict__ links, Geom g, float kappa,
                                                       DiagList dl, const int* __restrict__ act, int nvec,
                                                       int anti, int order) {
    __shared__ float2 sp[12 * 256];
    __shared__ float2 hl[8 * 6 * 64];
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const TileGeo tg(g, tile_of(g, (nb % 8 == 0) ? ((b % 8) * (nb / 8) + b / 8) : b, order));
    const int local = threadIdx.x;
    const int site0 = (tg.T << 8) | local;
    const int64_t V = g.vol;
    Z<float> ul[8][3][3];
    auto ldh = [&](auto muc, auto dirc) {
        constexpr int mu = decltype(muc)::value;
        constexpr int dir = decltype(dirc)::value;
        int ls;
        float sg;
        hop_link<mu, dir>(tg, local, anti, ls, sg);
        Z<float>(&u)[3][3] = ul[2 * mu + dir];
        ld_r12(links + (int64_t)mu * 6 * V, V, ls, u);
        // the boundary sign folded into the register copy of the link
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) u[a][bb] = {sg * u[a][bb].x, sg * u[a][bb].y};
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    ldh(I0{}, I0{});
    ldh(I0{}, I1{});
    ldh(I1{}, I0{});
    ldh(I1{}, I1{});
    ldh(I2{}, I0{});
    ldh(I2{}, I1{});
    ldh(I3{}, I0{});
    ldh(I3{}, I1{});
    bool first = true;
    for (int v = 0; v < nvec; ++v) {
        if (act && !act[v]) continue;   // uniform over the block
        if (!first) __syncthreads();   // the previous vector's LDS reads are done
        first = false;
        const int hsrc[2] = {halo_source(tg, local), halo_source(tg, local + 256)};
        stage_r12<true>(in + v * in_stride, V, site0, local, hsrc, sp, hl);
        __syncthreads();
        Z<float> acc[4][3];
#pragma unroll
        for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
            for (int a = 0; a < 3; ++a) acc[s_][a] = {0, 0};
        auto hop = [&](auto muc, auto dirc) {
            constexpr int mu = decltype(muc)::value;
            constexpr int dir = decltype(dirc)::value;
            int w = local;
            pin(w);
            Z<float> h0[3], h1[3];
            hop_input<mu, dir>(sp, hl, w, h0, h1);
            mulrec_sg<mu, dir>(acc, h0, h1, ul[2 * mu + dir], 1.f);
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    pin(acc[s_][a].x);
                    pin(acc[s_][a].y);
                }
        };
        hop(I0{}, I0{});
        hop(I0{}, I1{});
        hop(I1{}, I0{});
        hop(I1{}, I1{});
        hop(I2{}, I0{});
        hop(I2{}, I1{});
        hop(I3{}, I0{});
        hop(I3{}, I1{});
        finish_r12(acc, sp, local, out + v * out_stride + site0, nullptr, V, (float)dl.d[v].x,
                   (float)dl.d[v].y, (float)dl.alpha[v], kappa);
    }
}

template <typename TL>
__global__ __launch_bounds__(256, 3) void k_dslash_halo(const float2* __restrict__ in, int64_t in_stride,
                                                        float2* __restrict__ out, int64_t out_stride,
                                                        const float2* __restrict__ add, int64_t add_stride,
                                                        const TL* __restrict__ links, Geom g, float kappa,
                                                        DiagList dl, const int* __restrict__ act, int nvec) {
    DslashHaloK<TL>::run(in, in_stride, out, out_stride, add, add_stride, links, g, kappa, dl, act, nvec);
}

template <typename TS> struct DslashOcc { static constexpr int waves = 4; };
template <> struct DslashOcc<double> { static constexpr int waves = 2; };

template <typename TS, typename TL, typename R>
__global__ __launch_bounds__(256, DslashOcc<TS>::waves) void k_dslash(const typename CT<TS>::t* __restrict__ in,
                                                int64_t in_stride, typename CT<TS>::t* __restrict__ out,
                                                int64_t out_stride,
                                                const typename CT<TS>::t* __restrict__ add,
                                                int64_t add_stride, const TL* __restrict__ links,
                                                Geom g, R kappa, DiagList dl,
                                                const int* __restrict__ act, int nvec) {
    DslashK<TS, TL, R>::run(in, in_stride, out, out_stride, add, add_stride, links, g, kappa, dl,
                            act, nvec);
}

template <typename TS>
void dslash(const typename CT<TS>::t* in, int64_t in_stride, typename CT<TS>::t* out,
            int64_t out_stride, const typename CT<TS>::t* add, int64_t add_stride,
            const void* links, int link_storage, const Geom& g, double kappa, const DiagList& dl,
            int nvec, hipStream_t st, const int* act, int anti) {
    dim3 grid(((g.vol + 255) / 256) * nvec);
    if constexpr (std::is_same<TS, float>::value) {
        if (link_storage == LINK_R12 || link_storage == LINK_R12H) {
            if (g.ltv != 8) throw std::invalid_argument("dslash: two-row links need 4^4 tiles");
            const bool h = link_storage == LINK_R12H;
            // tuned choices (identical results): tile order, and for several
            // vectors the vector-loop kernel or one block per tile and vector
            const bool zt = g.nt[2] % 2 == 0 && g.nt[3] % 2 == 0;
            const bool loop = nvec >= DSLASH_VLOOP_MIN && !add;
            const int norder = zt ? 2 : 1;
            char shape[96];
            std::snprintf(shape, sizeof shape, "%dx%dx%dx%d|%d|%d", g.L[0], g.L[1], g.L[2], g.L[3],
                          nvec, add ? 1 : 0);
            TuneScope ts(h ? "dslash_r12h" : "dslash_r12", shape, loop ? 2 * norder : norder, 0, st);
            const int order = ts.choice() % norder;
#define R12_LAUNCH(LT)                                                                             \
    do {                                                                                           \
        if (loop && ts.choice() < norder)                                                          \
            hipLaunchKernelGGL(k_dslash_r12v<LT>, dim3(g.vol >> 8), dim3(256), 0, st, in,          \
                               in_stride, out, out_stride, (const LT*)links, g, (float)kappa, dl,  \
                               act, nvec, anti, order);                                            \
        else                                                                                       \
            hipLaunchKernelGGL(k_dslash_r12<LT>, grid, dim3(256), 0, st, in, in_stride, out,       \
                               out_stride, add, add_stride, (const LT*)links, g, (float)kappa, dl, \
                               act, nvec, anti, order);                                            \
    } while (0)
            if (h) R12_LAUNCH(__half2);
            else R12_LAUNCH(float2);
#undef R12_LAUNCH
            return;
        }
    }
    if constexpr (std::is_same<TS, double>::value) {
        hipLaunchKernelGGL((k_dslash<double, double2, double>), grid, dim3(256), 0, st, in,
                           in_stride, out, out_stride, add, add_stride, (const double2*)links, g,
                           kappa, dl, act, nvec);
    } else if (g.ltv == 8) {   // 4^4 tiles: halo-staged kernel
        if (link_storage == 2) {
            hipLaunchKernelGGL((k_dslash_halo<__half2>), grid, dim3(256), 0, st, in, in_stride, out,
                               out_stride, add, add_stride, (const __half2*)links, g, (float)kappa,
                               dl, act, nvec);
        } else {
            hipLaunchKernelGGL((k_dslash_halo<float2>), grid, dim3(256), 0, st, in, in_stride, out,
                               out_stride, add, add_stride, (const float2*)links, g, (float)kappa,
                               dl, act, nvec);
        }
    } else {
        if (link_storage == 2) {
            hipLaunchKernelGGL((k_dslash<float, __half2, float>), grid, dim3(256), 0, st, in,
                               in_stride, out, out_stride, add, add_stride,
                               (const __half2*)links, g, (float)kappa, dl, act, nvec);
        } else {
            hipLaunchKernelGGL((k_dslash<float, float2, float>), grid, dim3(256), 0, st, in,
                               in_stride, out, out_stride, add, add_stride, (const float2*)links,
                               g, (float)kappa, dl, act, nvec);
        }
    }
}

void dslash_list(const float2* in, int64_t in_stride, float2* out, int64_t out_stride,
                 const LatList& L, int link_storage, const DiagList& dl, hipStream_t st,
                 const int* act, int max_blocks) {
    if (L.nm < 1 || L.nm > DSLASH_MAXV) throw std::invalid_argument("dslash_list: 1..16 members");
    for (int v = 0; v < L.nm; ++v)
        if (L.g[v].ltv != 8 || L.tile0[v + 1] - L.tile0[v] != (L.g[v].vol >> 8))
            throw std::invalid_argument("dslash_list: members need 4^4 tiles and matching tile counts");
    const int total = L.tile0[L.nm];
    const int grid = total < max_blocks ? total : max_blocks;
    if (link_storage == LINK_R12H)
        hipLaunchKernelGGL(k_dslash_r12_list<__half2>, dim3(grid), dim3(256), 0, st, in, in_stride,
                           out, out_stride, L, dl, act);
    else if (link_storage == LINK_R12)
        hipLaunchKernelGGL(k_dslash_r12_list<float2>, dim3(grid), dim3(256), 0, st, in, in_stride,
                           out, out_stride, L, dl, act);
    else
        throw std::invalid_argument("dslash_list: two-row links only");
}

template void dslash<double>(const double2*, int64_t, double2*, int64_t, const double2*, int64_t,
                             const void*, int, const Geom&, double, const DiagList&, int,
                             hipStream_t, const int*, int);
template void dslash<float>(const float2*, int64_t, float2*, int64_t, const float2*, int64_t,
                            const void*, int, const Geom&, double, const DiagList&, int,
                            hipStream_t, const int*, int);

}  // namespace gdr
