// Internal definitions shared by the HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>

namespace gdr {

// Lattice geometry. Internal vectors are even-odd SoA: component c (spin*3 +
// colour, 0..11) of the site with checkerboard index s on parity p lives at
// [(p*12 + c)*vh + s]; links at [((p*4 + mu)*9 + a*3 + b)*vh + s] with the
// boundary factor bc[mu] folded into U_mu(x) on the last slice x_mu = L-1.
struct Geom {
    int L[4];   // Lx, Ly, Lz, Lt (all even)
    int vol;    // sites
    int vh;     // sites per parity
    int hx;     // Lx / 2
};

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
constexpr int MAXK = 63;
constexpr int CGS_GROUP = 16;             // columns reduced together
constexpr int CGS_MAXG = 5;               // up to 80 reduced columns
constexpr int CGS_BLOCK = 256;
constexpr int BASIS_PAD = 8;              // spare zeroed columns after every basis

}  // namespace gdr
