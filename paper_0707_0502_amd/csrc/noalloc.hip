// gdr_op_apply_noalloc: the operator application y_v = (A - sigma I) x_v of
// gdr_op_apply without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc). The two internal-layout staging buffers that
// gdr_op_apply takes from the context's cache live instead in one static
// device array of NOALLOC_BYTES per GPU (held until the process ends).
//
// In host code the array's name only stands for the device symbol: its device
// address is looked up once per device with hipGetSymbolAddress (at context
// creation, with the device current) and only that address is used.
#include <cmath>
#include <mutex>
#include <string>

#include "engine.h"

namespace gdr {
namespace {

constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int NOALLOC_MAXDEV = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

std::mutex g_mu;
void* g_ptr[NOALLOC_MAXDEV];      // device address of `scratch` per device
bool g_done[NOALLOC_MAXDEV];

}  // namespace

int noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAXDEV) return GDR_ERR_ARG;
    std::lock_guard<std::mutex> g(g_mu);
    if (g_done[device]) return g_ptr[device] ? GDR_OK : GDR_ERR_HIP;
    g_done[device] = true;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        g_ptr[device] = nullptr;
        return GDR_ERR_HIP;
    }
    g_ptr[device] = p;
    return GDR_OK;
}

static void* noalloc_ptr(int device) {
    if (device < 0 || device >= NOALLOC_MAXDEV) return nullptr;
    std::lock_guard<std::mutex> g(g_mu);
    return g_ptr[device];
}

// vectors per chunk that fit the workspace: an input and an output buffer of
// `chunk` internal-layout vectors, the second at a 256-byte aligned offset
static int64_t noalloc_chunk(int64_t n, size_t elem, int nvec) {
    const size_t per = (size_t)n * elem;
    const size_t per_al = (per + 255) / 256 * 256;
    if (2 * per_al > NOALLOC_BYTES) return 0;
    int64_t c = (int64_t)(NOALLOC_BYTES / (2 * per_al));
    if (c > DSLASH_MAXV) c = DSLASH_MAXV;
    if (c > nvec) c = nvec;
    return c;
}

template <typename T>
static void apply_chunks(gdr_op_s* op, const double2* x, double2* y, int nvec, double2 sig,
                         void* ws, hipStream_t st) {
    using C = typename CT<T>::t;
    const int64_t n = op->n;
    const int chunk = (int)noalloc_chunk(n, sizeof(C), nvec);
    const size_t off = ((size_t)chunk * n * sizeof(C) + 255) / 256 * 256;
    C* a = (C*)ws;
    C* b = (C*)((unsigned char*)ws + off);
    DiagList dl{};
    for (int v = 0; v < DSLASH_MAXV; ++v) {
        dl.d[v] = make_double2(1.0 - sig.x, -sig.y);
        dl.alpha[v] = 1;
    }
    for (int v0 = 0; v0 < nvec; v0 += chunk) {
        const int nb = std::min(chunk, nvec - v0);
        op_pack<T>(op, x + (int64_t)v0 * n, a, n, nb, st);
        op_apply<T>(op, a, n, b, n, nullptr, 0, dl, nb, st);
        op_unpack<T>(op, b, n, y + (int64_t)v0 * n, nb, st);
    }
}

}  // namespace gdr

using namespace gdr;

extern "C" int gdr_op_apply_noalloc(gdr_op op, gdr_c64 sigma, const gdr_c64* x, gdr_c64* y,
                                    int nvec, int precision) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    auto fail = [&](int code, const std::string& m) {
        c->err = m;
        return code;
    };
    if (!x || !y || nvec < 0) return fail(GDR_ERR_ARG, "null vector or negative nvec");
    if (precision != GDR_PREC_F64 && precision != GDR_PREC_F32)
        return fail(GDR_ERR_ARG, "precision must be F64 or F32");
    if (!std::isfinite(sigma.re) || !std::isfinite(sigma.im))
        return fail(GDR_ERR_ARG, "sigma is not finite");
    if (nvec == 0) return GDR_OK;
    const size_t elem = precision == GDR_PREC_F64 ? sizeof(double2) : sizeof(float2);
    if (noalloc_chunk(op->n, elem, nvec) < 1)
        return fail(GDR_ERR_ARG,
                    "operator too large for the static workspace: n = " + std::to_string(op->n) +
                        " exceeds " + std::to_string(NOALLOC_BYTES / 2 / elem) +
                        " unknowns at this precision (64 MiB holds an input and an output vector)");
    if (!device_ptr(x, c->device) || !device_ptr(y, c->device))
        return fail(GDR_ERR_ARG, "x and y must be device memory of the context's device");
    void* ws = noalloc_ptr(c->device);
    if (!ws) return fail(GDR_ERR_HIP, "static workspace of this device has no address");
    try {
        HIPCHK(hipSetDevice(c->device));
        const double2 s = make_double2(sigma.re, sigma.im);
        if (precision == GDR_PREC_F64)
            apply_chunks<double>(op, (const double2*)x, (double2*)y, nvec, s, ws, c->st);
        else
            apply_chunks<float>(op, (const double2*)x, (double2*)y, nvec, s, ws, c->st);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(c->st));
    } catch (const GdrError& e) {
        (void)hipStreamSynchronize(c->st);
        return fail(e.code, e.what());
    }
    return GDR_OK;
}
