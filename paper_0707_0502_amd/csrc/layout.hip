// Canonical <-> tile-blocked SoA layout conversion, link packing and the
// even-odd lattice tables (checked bit for bit against the oracle's tables).
#include "kernels.h"

namespace gdr {

__device__ __forceinline__ void lex_coords(const Geom& g, int lex, int& x, int& y, int& z, int& t) {
    x = lex % g.L[0];
    int r = lex / g.L[0];
    y = r % g.L[1];
    r /= g.L[1];
    z = r % g.L[2];
    t = r / g.L[2];
}

__device__ __forceinline__ int lex_of(const Geom& g, int x, int y, int z, int t) {
    return x + g.L[0] * (y + g.L[1] * (z + g.L[2] * t));
}

__device__ __forceinline__ int eo_of(const Geom& g, int lex, int x, int y, int z, int t) {
    int p = (x + y + z + t) & 1;
    return p * g.vh + (lex >> 1);
}

template <typename T>
__global__ void k_pack_spinor(const double2* __restrict__ canon, typename CT<T>::t* __restrict__ dst,
                              int64_t stride, Geom g) {
    int lex = blockIdx.x * blockDim.x + threadIdx.x;
    int v = blockIdx.y;
    if (lex >= g.vol) return;
    int c[4];
    lex_coords(g, lex, c[0], c[1], c[2], c[3]);
    const double2* src = canon + ((int64_t)v * g.vol + lex) * 12;
    typename CT<T>::t* d = dst + v * stride + site_of(g, c);
#pragma unroll
    for (int k = 0; k < 12; ++k) d[(int64_t)k * g.vol] = from_d<T>(src[k]);
}

template <typename T>
__global__ void k_unpack_spinor(const typename CT<T>::t* __restrict__ src, int64_t stride,
                                double2* __restrict__ canon, Geom g) {
    int lex = blockIdx.x * blockDim.x + threadIdx.x;
    int v = blockIdx.y;
    if (lex >= g.vol) return;
    int c[4];
    lex_coords(g, lex, c[0], c[1], c[2], c[3]);
    const typename CT<T>::t* s = src + v * stride + site_of(g, c);
    double2* d = canon + ((int64_t)v * g.vol + lex) * 12;
#pragma unroll
    for (int k = 0; k < 12; ++k) d[k] = to_d(s[(int64_t)k * g.vol]);
}

template <typename T>
void pack_spinor(const double2* canon, typename CT<T>::t* dst, int64_t stride, const Geom& g,
                 int nvec, hipStream_t st) {
    dim3 grid((g.vol + 255) / 256, nvec);
    hipLaunchKernelGGL(k_pack_spinor<T>, grid, dim3(256), 0, st, canon, dst, stride, g);
}
template <typename T>
void unpack_spinor(const typename CT<T>::t* src, int64_t stride, double2* canon, const Geom& g,
                   int nvec, hipStream_t st) {
    dim3 grid((g.vol + 255) / 256, nvec);
    hipLaunchKernelGGL(k_unpack_spinor<T>, grid, dim3(256), 0, st, src, stride, canon, g);
}
template void pack_spinor<double>(const double2*, double2*, int64_t, const Geom&, int, hipStream_t);
template void pack_spinor<float>(const double2*, float2*, int64_t, const Geom&, int, hipStream_t);
template void unpack_spinor<double>(const double2*, int64_t, double2*, const Geom&, int, hipStream_t);
template void unpack_spinor<float>(const float2*, int64_t, double2*, const Geom&, int, hipStream_t);

struct BC4 {
    int v[4];
};

// links internal: [mu][e = a*3+b][vol] in tile order, bc[mu] folded into
// U_mu(x) at x_mu = L_mu - 1. Storage 3 (FP32, special unitary links): rows
// 0 and 1 only, [mu][e = a*3+b, a < 2][vol], boundary factors not folded (the
// third row is rebuilt as conj(row0 x row1), which holds for det U = 1 only;
// the operator applies bc[mu] itself)
__global__ void k_pack_links(const double2* __restrict__ canon, void* __restrict__ out, int storage,
                             Geom g, BC4 bc) {
    int lex = blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= g.vol) return;
    int c[4];
    lex_coords(g, lex, c[0], c[1], c[2], c[3]);
    const int s = site_of(g, c);
    if (storage == 3 || storage == 4) {
        for (int mu = 0; mu < 4; ++mu) {
            const double2* src = canon + ((int64_t)mu * g.vol + lex) * 9;
            for (int e = 0; e < 6; ++e) {
                const int64_t o = ((int64_t)mu * 6 + e) * g.vol + s;
                if (storage == 3) ((float2*)out)[o] = make_float2((float)src[e].x, (float)src[e].y);
                else ((__half2*)out)[o] = __floats2half2_rn((float)src[e].x, (float)src[e].y);
            }
        }
        return;
    }
    for (int mu = 0; mu < 4; ++mu) {
        double f = (c[mu] == g.L[mu] - 1) ? (double)bc.v[mu] : 1.0;
        const double2* src = canon + ((int64_t)mu * g.vol + lex) * 9;
        int64_t base = ((int64_t)mu * 9) * g.vol + s;
        for (int e = 0; e < 9; ++e) {
            double2 u = cscale(src[e], f);
            int64_t o = base + (int64_t)e * g.vol;
            if (storage == 0) {
                ((double2*)out)[o] = u;
            } else if (storage == 1) {
                ((float2*)out)[o] = make_float2((float)u.x, (float)u.y);
            } else {
                ((__half2*)out)[o] = __floats2half2_rn((float)u.x, (float)u.y);
            }
        }
    }
}

// Largest deviation of the canonical links from SU(3) over the lattice:
// max(|U U^H - I|_max, |det U - 1|) per link, as the bit pattern of a
// non-negative double (monotone as an unsigned integer) in *dev_bits.
__global__ void k_su3_dev(const double2* __restrict__ canon, int64_t nlinks,
                          unsigned long long* __restrict__ dev_bits) {
    double worst = 0;
    for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < nlinks;
         l += (int64_t)gridDim.x * blockDim.x) {
        const double2* u = canon + l * 9;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double2 acc = mk(i == j ? -1.0 : 0.0, 0);
                for (int k = 0; k < 3; ++k) acc = cadd(acc, cmul(u[i * 3 + k], cconj(u[j * 3 + k])));
                worst = fmax(worst, cabs(acc));
            }
        // det by the first row's cofactors
        const double2 c0 = csub(cmul(u[4], u[8]), cmul(u[5], u[7]));
        const double2 c1 = csub(cmul(u[5], u[6]), cmul(u[3], u[8]));
        const double2 c2 = csub(cmul(u[3], u[7]), cmul(u[4], u[6]));
        const double2 det = cadd(cadd(cmul(u[0], c0), cmul(u[1], c1)), cmul(u[2], c2));
        worst = fmax(worst, cabs(csub(det, mk(1, 0))));
        if (!(worst == worst)) worst = 1e300;   // NaN entries count as far from SU(3)
    }
    atomicMax(dev_bits, (unsigned long long)__double_as_longlong(worst));
}

void su3_deviation(const double2* canon, int64_t nlinks, unsigned long long* dev_bits,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_su3_dev, dim3(1024), dim3(256), 0, st, canon, nlinks, dev_bits);
}

void pack_links(const double2* canon, void* out, int storage, const Geom& g, const int bc[4],
                hipStream_t st) {
    BC4 b{{bc[0], bc[1], bc[2], bc[3]}};
    hipLaunchKernelGGL(k_pack_links, dim3((g.vol + 255) / 256), dim3(256), 0, st, canon, out,
                       storage, g, b);
}

__global__ void k_tables(int32_t* __restrict__ eo_of_lex, int32_t* __restrict__ nbr,
                         int8_t* __restrict__ sign, Geom g) {
    int lex = blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= g.vol) return;
    int c[4];
    lex_coords(g, lex, c[0], c[1], c[2], c[3]);
    int eo = eo_of(g, lex, c[0], c[1], c[2], c[3]);
    eo_of_lex[lex] = eo;
    for (int d = 0; d < 8; ++d) {
        int mu = d & 3;
        int step = d < 4 ? 1 : -1;
        int cc[4] = {c[0], c[1], c[2], c[3]};
        cc[mu] += step;
        int8_t sg = 1;
        if (cc[mu] == g.L[mu]) {
            cc[mu] = 0;
            if (mu == 3) sg = -1;
        } else if (cc[mu] < 0) {
            cc[mu] = g.L[mu] - 1;
            if (mu == 3) sg = -1;
        }
        int nl = lex_of(g, cc[0], cc[1], cc[2], cc[3]);
        nbr[(int64_t)eo * 8 + d] = eo_of(g, nl, cc[0], cc[1], cc[2], cc[3]);
        sign[(int64_t)eo * 8 + d] = sg;
    }
}

void build_tables(int32_t* eo_of_lex, int32_t* nbr, int8_t* sign, const Geom& g, int bc_t,
                  hipStream_t st) {
    (void)bc_t;
    hipLaunchKernelGGL(k_tables, dim3((g.vol + 255) / 256), dim3(256), 0, st, eo_of_lex, nbr,
                       sign, g);
}

}  // namespace gdr
