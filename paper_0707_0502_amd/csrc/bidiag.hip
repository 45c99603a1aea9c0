// The bidiagonal test matrix of the paper's Examples 1-6 as a second
// operator: M has the diagonal d_0..d_{n-1} and the superdiagonal
// e_0..e_{n-2} (Example 1: d = 0.1, 1, 2, ..., n-1, e = 1). Vectors are plain
// complex arrays (canonical and internal layouts coincide).
//   out = alpha * (M in - sigma in) [+ add],   sigma = 1 - d_v of the DiagList
// (the same interface as the Wilson operator, whose diagonal part is 1 - sigma).
#include "kernels.h"

namespace gdr {

template <typename T>
__global__ __launch_bounds__(256) void k_bidiag(const typename CT<T>::t* __restrict__ in,
                                                int64_t in_stride,
                                                typename CT<T>::t* __restrict__ out,
                                                int64_t out_stride,
                                                const typename CT<T>::t* __restrict__ add,
                                                int64_t add_stride,
                                                const typename CT<T>::t* __restrict__ de, int64_t n,
                                                DiagList dl, const int* __restrict__ act) {
    using C = typename CT<T>::t;
    const int v = blockIdx.y;
    if (act && !act[v]) return;
    const C* x = in + v * in_stride;
    C* y = out + v * out_stride;
    const C* a = add ? add + v * add_stride : nullptr;
    const double2 shift = mk(dl.d[v].x - 1.0, dl.d[v].y);   // -sigma
    const double al = dl.alpha[v];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 xi = to_d(x[i]);
        double2 r = cmul(cadd(to_d(de[i]), shift), xi);
        if (i + 1 < n) r = cadd(r, cmul(to_d(de[n + i]), to_d(x[i + 1])));
        r = cscale(r, al);
        if (a) r = cadd(r, to_d(a[i]));
        y[i] = from_d<T>(r);
    }
}

template <typename T>
void bidiag_apply(const typename CT<T>::t* in, int64_t in_stride, typename CT<T>::t* out,
                  int64_t out_stride, const typename CT<T>::t* add, int64_t add_stride,
                  const typename CT<T>::t* de, int64_t n, const DiagList& dl, int nvec,
                  hipStream_t st, const int* act) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_bidiag<T>, dim3((unsigned)g, nvec), dim3(256), 0, st, in, in_stride, out,
                       out_stride, add, add_stride, de, n, dl, act);
}
template void bidiag_apply<double>(const double2*, int64_t, double2*, int64_t, const double2*,
                                   int64_t, const double2*, int64_t, const DiagList&, int,
                                   hipStream_t, const int*);
template void bidiag_apply<float>(const float2*, int64_t, float2*, int64_t, const float2*, int64_t,
                                  const float2*, int64_t, const DiagList&, int, hipStream_t,
                                  const int*);

// plain conversion between the canonical complex128 vectors and type T
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_plain_copy(const typename CT<TI>::t* __restrict__ x,
                                                    int64_t x_stride,
                                                    typename CT<TO>::t* __restrict__ y,
                                                    int64_t y_stride, int64_t n) {
    const int v = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        y[v * y_stride + i] = from_d<TO>(to_d(x[v * x_stride + i]));
}

template <typename TI, typename TO>
void plain_copy(const typename CT<TI>::t* x, int64_t x_stride, typename CT<TO>::t* y,
                int64_t y_stride, int64_t n, int nvec, hipStream_t st) {
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL((k_plain_copy<TI, TO>), dim3((unsigned)g, nvec), dim3(256), 0, st, x,
                       x_stride, y, y_stride, n);
}
template void plain_copy<double, double>(const double2*, int64_t, double2*, int64_t, int64_t, int,
                                         hipStream_t);
template void plain_copy<double, float>(const double2*, int64_t, float2*, int64_t, int64_t, int,
                                        hipStream_t);
template void plain_copy<float, double>(const float2*, int64_t, double2*, int64_t, int64_t, int,
                                        hipStream_t);

}  // namespace gdr
