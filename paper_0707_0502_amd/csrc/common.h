// Internal definitions shared by the HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

namespace gdr {

// Lattice geometry. Internal vectors are tile-blocked SoA: the lattice is cut
// into tiles of b_0 x b_1 x b_2 x b_3 sites (b_mu = 4 where L_mu is a multiple
// of 4, else 2), tiles are numbered lexicographically (x fastest) and the
// sites of a tile are stored contiguously, also lexicographically. Component c
// (spin*3 + colour, 0..11) of site s lives at [c*vol + s]; links at
// [(mu*9 + a*3 + b)*vol + s] with the boundary factor bc[mu] folded into
// U_mu(x) on the last slice x_mu = L_mu - 1. The even-odd numbering is kept
// for the lattice tables only.
struct Geom {
    int L[4];    // Lx, Ly, Lz, Lt (all even)
    int vol;     // sites
    int vh;      // sites per parity
    int hx;      // Lx / 2
    int lb[4];   // log2 of the tile extent per direction (1 or 2)
    int off[4];  // bit offset of direction mu inside the in-tile index
    int nt[4];   // tiles per direction
    int ltv;     // log2 of the tile volume
};

inline Geom make_geom(const int dims[4]) {
    Geom g;
    long long vol = 1;
    int o = 0;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = dims[mu];
        vol *= dims[mu];
        g.lb[mu] = dims[mu] % 4 == 0 ? 2 : 1;
        g.off[mu] = o;
        o += g.lb[mu];
        g.nt[mu] = dims[mu] >> g.lb[mu];
    }
    g.ltv = o;
    g.vol = (int)vol;
    g.vh = (int)(vol / 2);
    g.hx = dims[0] / 2;
    return g;
}

// storage index of the site with coordinates c[0..3]
__host__ __device__ __forceinline__ int site_of(const Geom& g, const int c[4]) {
    int tile = 0, w = 0;
#pragma unroll
    for (int mu = 3; mu >= 0; --mu) {
        tile = tile * g.nt[mu] + (c[mu] >> g.lb[mu]);
        w |= (c[mu] & ((1 << g.lb[mu]) - 1)) << g.off[mu];
    }
    return (tile << g.ltv) | w;
}

template <typename T> struct CT;
template <> struct CT<double> { using t = double2; };
template <> struct CT<float> { using t = float2; };

__host__ __device__ __forceinline__ double2 mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ __forceinline__ double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
__host__ __device__ __forceinline__ double2 cjmul(double2 a, double2 b) {
    return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__host__ __device__ __forceinline__ double2 cconj(double2 a) { return mk(a.x, -a.y); }
__host__ __device__ __forceinline__ double2 cscale(double2 a, double s) { return mk(a.x * s, a.y * s); }
__host__ __device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    // Smith's algorithm
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
    } else {
        double r = b.x / b.y, d = b.x * r + b.y;
        return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
    }
}
__host__ __device__ __forceinline__ double cabs(double2 a) { return hypot(a.x, a.y); }

__device__ __forceinline__ double2 to_d(double2 a) { return a; }
__device__ __forceinline__ double2 to_d(float2 a) { return mk((double)a.x, (double)a.y); }
template <typename T> __device__ __forceinline__ typename CT<T>::t from_d(double2 a);
template <> __device__ __forceinline__ double2 from_d<double>(double2 a) { return a; }
template <> __device__ __forceinline__ float2 from_d<float>(double2 a) {
    return make_float2((float)a.x, (float)a.y);
}

// Small sizes
constexpr int MAXM = 64;     // max restart length m
constexpr int MAXNS = 16;    // max shifts
constexpr int BLK_MAX = 8;   // max block of the s-step Arnoldi cycle
// block update coefficients per member: coef[o*(MAXM+1) + c], beta[o][a] after them
constexpr int BLK_COEF_MS = BLK_MAX * (MAXM + 1) + BLK_MAX * BLK_MAX;
constexpr int MAXK = 63;
constexpr int BASIS_PAD = 8;              // spare zeroed columns after every basis

}  // namespace gdr
