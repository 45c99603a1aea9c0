// The C-ABI of include/gdr.h: argument checks, canonical <-> internal layout
// conversion at the boundary, and error reporting.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>

#include "engine.h"
#include "tune.h"

using namespace gdr;

namespace {

int fail(gdr_ctx_s* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    return code;
}

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double sec() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

bool check_params(gdr_ctx_s* c, const gdr_params* p, int ns, bool need_dr) {
    if (!p) {
        c->err = "params is NULL";
        return false;
    }
    if (ns < 1 || ns > MAXNS) {
        c->err = "ns must be in 1..16";
        return false;
    }
    if (need_dr && !(p->m_dr >= 1 && p->m_dr <= MAXM && p->k >= 0 && p->k < p->m_dr)) {
        c->err = "need 0 <= k < m_dr <= 64";
        return false;
    }
    if (!(p->m_proj >= 1 && p->m_proj <= MAXM)) {
        c->err = "need 1 <= m_proj <= 64";
        return false;
    }
    if (p->m_clean < 0 || p->m_clean > MAXM) {
        c->err = "need 0 <= m_clean <= 64";
        return false;
    }
    if (!(p->refine_floor >= 0 && p->refine_floor <= 0.5)) {
        c->err = "need 0 <= refine_floor <= 0.5";
        return false;
    }
    if (p->proj_k < 0 || p->proj_k > p->k) {
        c->err = "need 0 <= proj_k <= k";
        return false;
    }
    if (p->use_graph != 0 && p->use_graph != 1) {
        c->err = "use_graph must be 0 or 1";
        return false;
    }
    if (p->galerkin != 0 && p->galerkin != 1) {
        c->err = "galerkin must be 0 or 1";
        return false;
    }
    if (p->sstep < 0 || p->sstep > BLK_MAX) {
        c->err = "need 0 <= sstep <= 8";
        return false;
    }
    if (!(p->sstep_reorth >= 0)) {
        c->err = "need sstep_reorth >= 0";
        return false;
    }
    if (!(p->tol > 0) || p->max_cycles < 1 || p->max_refine < 0) {
        c->err = "need tol > 0, max_cycles >= 1, max_refine >= 0";
        return false;
    }
    if (p->precision != GDR_PREC_F64 && p->precision != GDR_PREC_MIXED) {
        c->err = "precision must be GDR_PREC_F64 or GDR_PREC_MIXED";
        return false;
    }
    if (p->persistent != 0 && p->persistent != 1) {
        c->err = "persistent must be 0 or 1";
        return false;
    }
    return true;
}

void stats_reset(gdr_stats* st) {
    if (!st) return;
    st->cycles_dr = st->cycles_extra = st->cycles_proj = st->cycles_cleanup = 0;
    st->mvp_dr = st->mvp_extra = st->mvp_proj = st->mvp_fp64 = st->mvp_cleanup = 0;
    st->t_total = 0;
    for (double& t : st->t_phase) t = 0;
    st->hist_len = 0;
    st->theta_len = 0;
    for (int i = 0; i < 8; ++i) {
        st->k_ms[i] = st->k_bytes[i] = st->k_flops[i] = 0;
        st->k_launches[i] = 0;
    }
    st->resid_main = 0;
}

bool finite_shifts(gdr_ctx_s* c, const gdr_c64* sigma, int ns) {
    for (int i = 0; i < ns; ++i)
        if (!std::isfinite(sigma[i].re) || !std::isfinite(sigma[i].im)) {
            c->err = "shift " + std::to_string(i) + " is not finite";
            return false;
        }
    return true;
}

// every right-hand side must have a finite norm (a NaN or Inf entry, or an
// overflowing norm, is rejected before any solve starts)
void check_rhs(gdr_op_s* op, const double2* Beo, int nrhs) {
    const std::vector<double> r = norms_of(op, Beo, nrhs);
    for (int j = 0; j < nrhs; ++j)
        if (!std::isfinite(r[j]))
            throw GdrError(GDR_ERR_ARG, "right-hand side " + std::to_string(j) +
                                            " is not finite (||b|| = " + std::to_string(r[j]) + ")");
}

template <typename T>
void dslash_bench_run(gdr_op op, int nvec, int nsets, int reps, double* ms_each) {
    using C = typename CT<T>::t;
    gdr_ctx_s* c = op->ctx;
    const int64_t n = op->n;
    DMem mem;
    std::vector<C*> xin(nsets), yout(nsets);
    for (int k = 0; k < nsets; ++k) {
        xin[k] = mem.get<C>((size_t)n * nvec);
        yout[k] = mem.get<C>((size_t)n * nvec);
        // a finite bit pattern: the timing does not depend on the values
        HIPCHK(hipMemsetAsync(xin[k], 0x3c, (size_t)n * nvec * sizeof(C), c->st));
    }
    DiagList dl{};
    for (int v = 0; v < DSLASH_MAXV; ++v) {
        dl.d[v] = make_double2(1, 0);
        dl.alpha[v] = 1;
    }
    // launches until the launch tuner has decided this shape (each waits for
    // its timing), so that the timed repetitions run the decided form
    for (int w = 0; w < TUNE_REPS * TUNE_MAXCAND + 1 && tune_active(); ++w) {
        op_apply<T>(op, xin[0], n, yout[0], n, nullptr, 0, dl, nvec, c->st);
        HIPCHK(hipStreamSynchronize(c->st));
    }
    std::vector<hipEvent_t> ev(2 * reps);
    for (auto& e : ev) HIPCHK(hipEventCreate(&e));
    try {
        for (int r = 0; r < reps; ++r) {
            const int k = r % nsets;
            HIPCHK(hipEventRecord(ev[2 * r], c->st));
            op_apply<T>(op, xin[k], n, yout[k], n, nullptr, 0, dl, nvec, c->st);
            HIPCHK(hipEventRecord(ev[2 * r + 1], c->st));
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(c->st));
        for (int r = 0; r < reps; ++r) {
            float t = 0;
            HIPCHK(hipEventElapsedTime(&t, ev[2 * r], ev[2 * r + 1]));
            ms_each[r] = t;
        }
    } catch (...) {
        for (auto& e : ev) (void)hipEventDestroy(e);
        throw;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
}

}  // namespace

#define API_TRY(c) try { gdr::PoolScope pool_scope_((c));
#define API_CATCH(c)                                                \
    }                                                               \
    catch (const GdrError& e) {                                     \
        (void)hipStreamSynchronize((c)->st);                        \
        return fail((c), e.code, e.what());                         \
    }                                                               \
    catch (const std::exception& e) {                               \
        return fail((c), GDR_ERR_HIP, e.what());                    \
    }

namespace gdr {
// A vector argument must be device memory of the context's device (or
// managed memory): a host pointer handed to a kernel would fault the GPU.
bool device_ptr(const void* p, int device) {
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    if (a.type == hipMemoryTypeUnregistered || a.type == hipMemoryTypeHost) return false;
    if (a.type == hipMemoryTypeDevice && a.device != device) return false;
    return true;
}
}  // namespace gdr

extern "C" {

int gdr_ctx_create(int device, void* hip_stream, gdr_ctx* out) {
    if (!out) return GDR_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return GDR_ERR_HIP;
    if (device < 0 || device >= ndev) return GDR_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return GDR_ERR_HIP;
    gdr_ctx_s* c = new gdr_ctx_s;
    c->device = device;
    c->st = (hipStream_t)hip_stream;
    if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        gdr_ctx_destroy(c);
        return GDR_ERR_HIP;
    }
    c->pool.attach(device);
    // the device address of gdr_op_apply_noalloc's static workspace
    if (noalloc_setup(device) != GDR_OK) {
        gdr_ctx_destroy(c);
        return GDR_ERR_HIP;
    }
    *out = c;
    return GDR_OK;
}

void gdr_ctx_destroy(gdr_ctx c) {
    if (!c) return;
    if (c->aux) {
        (void)hipStreamSynchronize(c->aux);
        (void)hipStreamDestroy(c->aux);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    for (hipEvent_t e : c->evpool) (void)hipEventDestroy(e);
    (void)hipStreamSynchronize(c->st);
    c->pool.detach();
    delete c;
}

const char* gdr_last_error(gdr_ctx c) { return c ? c->err.c_str() : "null context"; }

void gdr_params_default(gdr_params* p) {
    if (!p) return;
    p->m_dr = 40;
    p->k = 15;
    p->m_proj = 40;
    p->tol = 1e-8;
    p->tol_extra = 0;
    p->max_cycles = 1000;
    p->precision = GDR_PREC_F64;
    p->batch = 1;
    p->related_rhs = 0;
    p->max_refine = 8;
    p->profile = 0;
    p->m_clean = 0;
    p->proj_k = 0;
    p->use_graph = 0;
    p->galerkin = 0;
    p->sstep = 8;
    p->sstep_reorth = 20;
    p->refine_floor = 0;
    p->persistent = 0;
}

int gdr_wilson_create(gdr_ctx c, const int dims[4], const int bc[4], double kappa,
                      const gdr_c64* links, int links_on_device, int link_storage, gdr_op* out) {
    if (!c) return GDR_ERR_ARG;
    if (!dims || !bc || !links || !out) return fail(c, GDR_ERR_ARG, "null argument");
    *out = nullptr;
    for (int mu = 0; mu < 4; ++mu) {
        if (dims[mu] < 2 || dims[mu] % 2) return fail(c, GDR_ERR_ARG, "lattice extents must be even and >= 2");
        if (bc[mu] != 1 && bc[mu] != -1) return fail(c, GDR_ERR_ARG, "bc must be +1 or -1");
    }
    if (link_storage < GDR_LINKS_F64 || link_storage > GDR_LINKS_F16)
        return fail(c, GDR_ERR_ARG, "link_storage must be F64, F32 or F16");
    if (!std::isfinite(kappa)) return fail(c, GDR_ERR_ARG, "kappa not finite");
    const int64_t vol = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
    if (vol > (int64_t)1 << 30) return fail(c, GDR_ERR_ARG, "lattice too large");
    if (links_on_device != 0 && links_on_device != 1)
        return fail(c, GDR_ERR_ARG, "links_on_device must be 0 or 1");
    if (links_on_device && !device_ptr(links, c->device))
        return fail(c, GDR_ERR_ARG, "links_on_device = 1 but links is not device memory of the context's device");
    gdr_op_s* op = new gdr_op_s;
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    op->ctx = c;
    for (int mu = 0; mu < 4; ++mu) op->bc[mu] = bc[mu];
    op->g = make_geom(dims);
    op->kappa = kappa;
    // A = I - kappa D with |lambda(D)| <= 8 for SU(3) links
    op->spec_c = make_double2(1, 0);
    op->spec_r = 8 * std::fabs(kappa) > 0 ? 8 * std::fabs(kappa) : 1;
    op->n = 12 * vol;
    op->lst = link_storage == GDR_LINKS_F64 ? GDR_LINKS_F32 : link_storage;
    for (int mu = 0; mu < 4; ++mu)
        if (bc[mu] == -1) op->anti |= 1 << mu;
    const size_t nl = (size_t)36 * vol;
    HIPCHK(hipMalloc(&op->u64, nl * sizeof(double2)));
    const double2* src = (const double2*)links;
    double2* tmp = nullptr;
    if (!links_on_device) {
        HIPCHK(hipMalloc(&tmp, nl * sizeof(double2)));
        HIPCHK(hipMemcpyAsync(tmp, links, nl * sizeof(double2), hipMemcpyHostToDevice, c->st));
        src = tmp;
    }
    bool su3 = false;
    if (op->g.ltv == 8) {
        // special unitary links (to 1e-9) are stored for the FP32 operator as
        // their first two rows; any other field keeps all nine entries
        DMem mem;
        unsigned long long* devb = mem.get<unsigned long long>(1);
        HIPCHK(hipMemsetAsync(devb, 0, sizeof(unsigned long long), c->st));
        su3_deviation(src, 4 * vol, devb, c->st);
        unsigned long long bits = 0;
        HIPCHK(hipMemcpyAsync(&bits, devb, sizeof(bits), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        double dev;
        std::memcpy(&dev, &bits, sizeof(dev));
        op->su3_dev = dev;
        su3 = dev <= 1e-9;
        if (su3 && op->lst == GDR_LINKS_F32) op->lst = LINK_R12;
        if (su3 && op->lst == GDR_LINKS_F16) op->lst = LINK_R12H;
    }
    const bool two_row = op->lst == LINK_R12 || op->lst == LINK_R12H;
    const bool fp16 = op->lst == GDR_LINKS_F16 || op->lst == LINK_R12H;
    const size_t nlo = two_row ? (size_t)24 * vol : nl;
    HIPCHK(hipMalloc(&op->ulo, nlo * (fp16 ? sizeof(__half2) : sizeof(float2))));
    pack_links(src, op->u64, GDR_LINKS_F64, op->g, bc, c->st);
    pack_links(src, op->ulo, op->lst, op->g, bc, c->st);
    if (fp16) {
        // FP32 copy for the refinement solves of the mixed-precision cleanup:
        // an inner solve on FP16-rounded links gains only about 1e-3 per round
        op->lre = su3 ? LINK_R12 : GDR_LINKS_F32;
        HIPCHK(hipMalloc(&op->ure, (su3 ? (size_t)24 * vol : nl) * sizeof(float2)));
        pack_links(src, op->ure, op->lre, op->g, bc, c->st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    if (tmp) (void)hipFree(tmp);
    *out = op;
    return GDR_OK;
    }
    catch (const GdrError& e) {
        if (op->u64) (void)hipFree(op->u64);
        if (op->ulo) (void)hipFree(op->ulo);
        if (op->ure) (void)hipFree(op->ure);
        delete op;
        return fail(c, e.code, e.what());
    }
}

void gdr_op_destroy(gdr_op op) {
    if (!op) return;
    if (op->u64) (void)hipFree(op->u64);
    if (op->ulo) (void)hipFree(op->ulo);
    if (op->ure) (void)hipFree(op->ure);
    if (op->bd64) (void)hipFree(op->bd64);
    if (op->bd32) (void)hipFree(op->bd32);
    delete op;
}

int gdr_bidiag_create(gdr_ctx c, int64_t n, const gdr_c64* diag, const gdr_c64* super,
                      gdr_op* out) {
    if (!c || !out) return GDR_ERR_ARG;
    *out = nullptr;
    if (n < 1 || n > ((int64_t)1 << 30)) return fail(c, GDR_ERR_ARG, "n must be 1..2^30");
    if (!diag || (n > 1 && !super)) return fail(c, GDR_ERR_ARG, "null diagonal or superdiagonal");
    std::vector<double2> h((size_t)2 * n, make_double2(0, 0));
    for (int64_t i = 0; i < n; ++i) {
        h[i] = make_double2(diag[i].re, diag[i].im);
        if (i + 1 < n) h[n + i] = make_double2(super[i].re, super[i].im);
    }
    for (const double2& v : h)
        if (!std::isfinite(v.x) || !std::isfinite(v.y))
            return fail(c, GDR_ERR_ARG, "matrix entries must be finite");
    gdr_op_s* op = new gdr_op_s;
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    op->ctx = c;
    op->kind = 1;
    op->n = n;
    {
        // Gershgorin: centre of the diagonal's bounding box, radius to the
        // farthest diagonal entry plus the largest superdiagonal modulus
        double xmin = h[0].x, xmax = h[0].x, ymin = h[0].y, ymax = h[0].y, emax = 0;
        for (int64_t i = 0; i < n; ++i) {
            xmin = std::min(xmin, h[i].x);
            xmax = std::max(xmax, h[i].x);
            ymin = std::min(ymin, h[i].y);
            ymax = std::max(ymax, h[i].y);
            if (i + 1 < n) emax = std::max(emax, std::hypot(h[n + i].x, h[n + i].y));
        }
        op->spec_c = make_double2(0.5 * (xmin + xmax), 0.5 * (ymin + ymax));
        double r = 0;
        for (int64_t i = 0; i < n; ++i)
            r = std::max(r, std::hypot(h[i].x - op->spec_c.x, h[i].y - op->spec_c.y));
        op->spec_r = r + emax > 0 ? r + emax : 1;
    }
    HIPCHK(hipMalloc(&op->bd64, (size_t)2 * n * sizeof(double2)));
    HIPCHK(hipMalloc(&op->bd32, (size_t)2 * n * sizeof(float2)));
    HIPCHK(hipMemcpyAsync(op->bd64, h.data(), (size_t)2 * n * sizeof(double2),
                          hipMemcpyHostToDevice, c->st));
    plain_copy<double, float>(op->bd64, 0, op->bd32, 0, 2 * n, 1, c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    *out = op;
    return GDR_OK;
    } catch (const GdrError& e) {
        gdr_op_destroy(op);
        return fail(c, e.code, e.what());
    } catch (const std::exception& e) {
        gdr_op_destroy(op);
        return fail(c, GDR_ERR_HIP, e.what());
    }
}

int64_t gdr_op_size(gdr_op op) { return op ? op->n : 0; }

int gdr_op_link_bytes(gdr_op op, int precision) {
    if (!op || op->kind != 0) return -1;
    if (precision == GDR_PREC_F64) return 4 * 9 * 16;
    if (precision != GDR_PREC_F32) return -1;
    return op->lst == LINK_R12    ? 4 * 6 * 8
           : op->lst == LINK_R12H ? 4 * 6 * 4
           : op->lst == GDR_LINKS_F16 ? 4 * 9 * 4
                                      : 4 * 9 * 8;
}

int gdr_op_apply(gdr_op op, gdr_c64 sigma, const gdr_c64* x, gdr_c64* y, int nvec, int precision) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    if (!x || !y || nvec < 0) return fail(c, GDR_ERR_ARG, "null vector or negative nvec");
    if (precision != GDR_PREC_F64 && precision != GDR_PREC_F32)
        return fail(c, GDR_ERR_ARG, "precision must be F64 or F32");
    if (nvec == 0) return GDR_OK;
    if (!device_ptr(x, c->device) || !device_ptr(y, c->device))
        return fail(c, GDR_ERR_ARG, "x and y must be device memory of the context's device");
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    const int64_t n = op->n;
    DMem mem;
    const int chunk = std::min(nvec, DSLASH_MAXV);
    DiagList dl{};
    for (int v = 0; v < DSLASH_MAXV; ++v) {
        dl.d[v] = make_double2(1.0 - sigma.re, -sigma.im);
        dl.alpha[v] = 1;
    }
    if (precision == GDR_PREC_F64) {
        double2* a = mem.get<double2>((size_t)chunk * n);
        double2* b = mem.get<double2>((size_t)chunk * n);
        for (int v0 = 0; v0 < nvec; v0 += chunk) {
            const int nb = std::min(chunk, nvec - v0);
            op_pack<double>(op, (const double2*)x + v0 * n, a, n, nb, c->st);
            op_apply<double>(op, a, n, b, n, nullptr, 0, dl, nb,
                           c->st);
            op_unpack<double>(op, b, n, (double2*)y + v0 * n, nb, c->st);
        }
    } else {
        float2* a = mem.get<float2>((size_t)chunk * n);
        float2* b = mem.get<float2>((size_t)chunk * n);
        for (int v0 = 0; v0 < nvec; v0 += chunk) {
            const int nb = std::min(chunk, nvec - v0);
            op_pack<float>(op, (const double2*)x + v0 * n, a, n, nb, c->st);
            op_apply<float>(op, a, n, b, n, nullptr, 0, dl, nb, c->st);
            op_unpack<float>(op, b, n, (double2*)y + v0 * n, nb, c->st);
        }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->st));
    return GDR_OK;
    API_CATCH(c)
}

int gdr_op_tables(gdr_op op, int32_t* eo_of_lex, int32_t* nbr, int8_t* sign) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    if (!eo_of_lex || !nbr || !sign) return fail(c, GDR_ERR_ARG, "null table buffer");
    if (op->kind != 0) return fail(c, GDR_ERR_ARG, "not a lattice operator");
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    DMem mem;
    const int64_t vol = op->g.vol;
    int32_t* e = mem.get<int32_t>(vol);
    int32_t* nb = mem.get<int32_t>(8 * vol);
    int8_t* sg = mem.get<int8_t>(8 * vol);
    build_tables(e, nb, sg, op->g, op->bc[3], c->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(eo_of_lex, e, vol * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(nbr, nb, 8 * vol * sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(sign, sg, 8 * vol, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return GDR_OK;
    API_CATCH(c)
}

int gdr_op_dslash_bench(gdr_op op, int precision, int nvec, int nsets, int reps,
                        double* ms_each) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    if (!ms_each) return fail(c, GDR_ERR_ARG, "null ms_each");
    if (nvec < 1 || nvec > DSLASH_MAXV) return fail(c, GDR_ERR_ARG, "nvec must be 1..16");
    if (nsets < 1 || nsets > 8) return fail(c, GDR_ERR_ARG, "nsets must be 1..8");
    if (reps < 1 || reps > 100000) return fail(c, GDR_ERR_ARG, "reps must be 1..100000");
    if (precision != GDR_PREC_F64 && precision != GDR_PREC_F32)
        return fail(c, GDR_ERR_ARG, "precision must be F64 or F32");
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    if (precision == GDR_PREC_F64)
        dslash_bench_run<double>(op, nvec, nsets, reps, ms_each);
    else
        dslash_bench_run<float>(op, nvec, nsets, reps, ms_each);
    return GDR_OK;
    API_CATCH(c)
}

// Final FP64 true residuals ||b - (A - sigma_i) x_i|| / ||b||: into the
// caller's array when there is one, and always in plain FP64, whose solves
// end on the method's own (recurrence) residuals and whose corrected shifts
// are only as accurate as the extra right-hand side; the mixed path's cleanup
// has already checked them. Returns the largest, or -1 if not computed.
static double finish_stats(gdr_op op, gdr_stats* st, int ns, const double2* sig, int nrhs,
                           const double2* Beo, const double2* Xeo, const Timer& t, int precision) {
    double rmax = -1;
    if ((st && st->resid) || precision == GDR_PREC_F64) {
        Timer tv;
        std::vector<double> r;
        true_residuals(op, ns, sig, nrhs, Beo, Xeo, r);
        // a NaN residual propagates (and fails every "<= tol" test)
        rmax = 0;
        for (double v : r)
            if (std::isnan(v) || v > rmax) rmax = v;
        if (st) {
            if (st->resid) std::memcpy(st->resid, r.data(), r.size() * sizeof(double));
            st->t_phase[5] += tv.sec();
            st->mvp_fp64 += (int64_t)ns * nrhs;
        }
    }
    if (st) st->t_total = t.sec();
    return rmax;
}

// vector arguments of the solvers: device memory of the context's device
static bool solve_ptrs_ok(gdr_ctx_s* c, const void* b, const void* x) {
    if (device_ptr(b, c->device) && device_ptr(x, c->device)) return true;
    c->err = "right-hand sides and solutions must be device memory of the context's device";
    return false;
}

// status of a finished solve: GDR_OK only if every final FP64 true residual
// is at most tol (a NaN residual is not)
static int final_status(int rc, double rmax, double tol) {
    return (rc == GDR_OK && !(rmax <= tol)) ? GDR_NOT_CONVERGED : rc;
}

int gdr_solve_dr_sh(gdr_op op, int ns, const gdr_c64* sigma, const gdr_c64* b, gdr_c64* x,
                    const gdr_params* p, gdr_stats* st, gdr_defl* defl_out) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    if (!sigma || !b || !x) return fail(c, GDR_ERR_ARG, "null argument");
    if (defl_out) *defl_out = nullptr;
    if (!check_params(c, p, ns, true) || !finite_shifts(c, sigma, ns) || !solve_ptrs_ok(c, b, x))
        return GDR_ERR_ARG;
    stats_reset(st);
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    Timer t;
    const int64_t n = op->n;
    DMem mem;
    double2* beo = mem.get<double2>(n);
    double2* Xeo = mem.get<double2>((size_t)ns * n);
    op_pack<double>(op, (const double2*)b, beo, n, 1, c->st);
    check_rhs(op, beo, 1);
    Stats S(st, (unsigned)p->profile, c->st, &c->evpool);
    gdr_defl_s* d = nullptr;
    // owns the deflation pair until it is handed to the caller (every error
    // path below releases it)
    struct Own {
        gdr_defl_s*& d;
        ~Own() { delete d; }
    } own{d};
    bool conv = false;
    Timer tdr;
    int rc = solve_dr_sh(op, ns, (const double2*)sigma, beo, Xeo, *p, S, &d, &conv);
    if (st) st->t_phase[0] += tdr.sec();
    if (p->precision == GDR_PREC_MIXED) {
        Timer tc;
        rc = cleanup(op, d, ns, (const double2*)sigma, 1, beo, Xeo, *p, S);
        if (st) st->t_phase[4] += tc.sec();
    }
    S.flush();
    rc = final_status(rc, finish_stats(op, st, ns, (const double2*)sigma, 1, beo, Xeo, t,
                                       p->precision),
                      p->tol);
    op_unpack<double>(op, Xeo, n, (double2*)x, ns, c->st);
    HIPCHK(hipStreamSynchronize(c->st));
    if (st) st->t_total = t.sec();
    if (defl_out) {
        *defl_out = d;
        d = nullptr;
    }
    return rc;
    API_CATCH(c)
}

int gdr_solve_proj_sh(gdr_op op, gdr_defl defl, int ns, const gdr_c64* sigma, int nrhs,
                      const gdr_c64* B, gdr_c64* X, const gdr_params* p, gdr_stats* st) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    if (!defl || !sigma || !B || !X || nrhs < 1) return fail(c, GDR_ERR_ARG, "null argument or nrhs < 1");
    if (defl->op != op) return fail(c, GDR_ERR_STATE, "deflation handle belongs to another operator");
    if (!check_params(c, p, ns, false) || !finite_shifts(c, sigma, ns) || !solve_ptrs_ok(c, B, X))
        return GDR_ERR_ARG;
    stats_reset(st);
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    Timer t;
    const int64_t n = op->n;
    DMem mem;
    double2* Beo = mem.get<double2>((size_t)nrhs * n);
    double2* Xeo = mem.get<double2>((size_t)nrhs * ns * n);
    op_pack<double>(op, (const double2*)B, Beo, n, nrhs, c->st);
    check_rhs(op, Beo, nrhs);
    Stats S(st, (unsigned)p->profile, c->st, &c->evpool);
    int rc = solve_proj_batch(op, defl, ns, (const double2*)sigma, nrhs, Beo, Xeo, 0, *p, S);
    if (p->precision == GDR_PREC_MIXED) {
        Timer tc;
        rc = cleanup(op, defl, ns, (const double2*)sigma, nrhs, Beo, Xeo, *p, S);
        if (st) st->t_phase[4] += tc.sec();
    }
    S.flush();
    rc = final_status(rc, finish_stats(op, st, ns, (const double2*)sigma, nrhs, Beo, Xeo, t,
                                       p->precision),
                      p->tol);
    op_unpack<double>(op, Xeo, n, (double2*)X, nrhs * ns, c->st);
    HIPCHK(hipStreamSynchronize(c->st));
    if (st) st->t_total = t.sec();
    return rc;
    API_CATCH(c)
}

int gdr_solve(gdr_op op, int ns, const gdr_c64* sigma, int nrhs, const gdr_c64* B, gdr_c64* X,
              const gdr_params* p, gdr_stats* st) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    if (!sigma || !B || !X || nrhs < 1) return fail(c, GDR_ERR_ARG, "null argument or nrhs < 1");
    if (!check_params(c, p, ns, true) || !finite_shifts(c, sigma, ns) || !solve_ptrs_ok(c, B, X))
        return GDR_ERR_ARG;
    stats_reset(st);
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    Timer t;
    const int64_t n = op->n;
    DMem mem;
    double2* Beo = mem.get<double2>((size_t)nrhs * n);
    double2* Xeo = mem.get<double2>((size_t)nrhs * ns * n);
    op_pack<double>(op, (const double2*)B, Beo, n, nrhs, c->st);
    check_rhs(op, Beo, nrhs);
    Stats S(st, (unsigned)p->profile, c->st, &c->evpool);
    gdr_defl_s* d = nullptr;
    struct Own {
        gdr_defl_s*& d;
        ~Own() { delete d; }
    } own{d};
    bool conv = false;
    Timer tdr;
    int rc = solve_dr_sh(op, ns, (const double2*)sigma, Beo, Xeo, *p, S, &d, &conv);
    HIPCHK(hipStreamSynchronize(c->st));
    if (st) st->t_phase[0] += tdr.sec();
    if (nrhs > 1) {
        if (!d) throw GdrError(GDR_ERR_BREAKDOWN, "first solve ended in a lucky breakdown: no deflation space");
        int rc2 = solve_proj_batch(op, d, ns, (const double2*)sigma, nrhs - 1, Beo + n,
                                   Xeo + (int64_t)ns * n, 1, *p, S);
        if (rc2 != GDR_OK) rc = rc2;
    }
    if (p->precision == GDR_PREC_MIXED) {
        Timer tc;
        rc = cleanup(op, d, ns, (const double2*)sigma, nrhs, Beo, Xeo, *p, S);
        if (st) st->t_phase[4] += tc.sec();
    }
    S.flush();
    rc = final_status(rc, finish_stats(op, st, ns, (const double2*)sigma, nrhs, Beo, Xeo, t,
                                       p->precision),
                      p->tol);
    op_unpack<double>(op, Xeo, n, (double2*)X, nrhs * ns, c->st);
    HIPCHK(hipStreamSynchronize(c->st));
    if (st) st->t_total = t.sec();
    return rc;
    API_CATCH(c)
}

int gdr_solve_many(int nops, const gdr_op* ops, int ns, const gdr_c64* sigma, int nrhs,
                   const gdr_c64* const* B, gdr_c64* const* X, const gdr_params* p, gdr_stats* st) {
    if (nops < 1 || !ops) return GDR_ERR_ARG;
    for (int l = 0; l < nops; ++l)
        if (!ops[l]) return GDR_ERR_ARG;
    gdr_ctx_s* c0 = ops[0]->ctx;
    if (!sigma || !B || !X || nrhs < 1 || !p)
        return fail(c0, GDR_ERR_ARG, "null argument or nrhs < 1");
    if (!check_params(c0, p, ns, true) || !finite_shifts(c0, sigma, ns)) return GDR_ERR_ARG;
    for (int l = 0; l < nops; ++l)
        if (!B[l] || !X[l] || !solve_ptrs_ok(ops[l]->ctx, B[l], X[l])) {
            if (ops[l]->ctx != c0) c0->err = ops[l]->ctx->err;
            return fail(c0, GDR_ERR_ARG, c0->err.empty() ? "null right-hand side or solution"
                                                         : c0->err.c_str());
        }
    if (!p->persistent) {
        // one lattice after another, each a gdr_solve on its own context
        int rc_all = GDR_OK;
        for (int l = 0; l < nops; ++l) {
            const int rc = gdr_solve(ops[l], ns, sigma, nrhs, B[l], X[l], p, st ? st + l : nullptr);
            if (rc < 0) return fail(c0, rc, gdr_last_error(ops[l]->ctx));
            if (rc != GDR_OK && rc_all == GDR_OK) rc_all = rc;
        }
        return rc_all;
    }
    // ---- one persistent batch for the first right-hand sides
    if (nops > DSLASH_MAXV) return fail(c0, GDR_ERR_ARG, "persistent: at most 16 lattices");
    if (p->precision != GDR_PREC_MIXED || p->sstep < 2)
        return fail(c0, GDR_ERR_ARG, "persistent: needs mixed precision and sstep >= 2");
    for (int l = 0; l < nops; ++l) {
        gdr_op_s* q = ops[l];
        if (q->kind != 0 || q->g.ltv != 8 || (q->lst != LINK_R12 && q->lst != LINK_R12H))
            return fail(c0, GDR_ERR_ARG, "persistent: every operator must be a Wilson operator "
                                         "with links stored as two rows (special unitary, extents "
                                         "multiples of 4)");
        if (q->lst != ops[0]->lst)
            return fail(c0, GDR_ERR_ARG, "persistent: all lattices need the same link precision");
        if (q->ctx->device != c0->device)
            return fail(c0, GDR_ERR_ARG, "persistent: all lattices on one device");
        for (int l2 = 0; l2 < l; ++l2)
            if (ops[l2] == q) return fail(c0, GDR_ERR_ARG, "persistent: an operator appears twice");
    }
    for (int l = 0; l < nops; ++l) stats_reset(st ? st + l : nullptr);
    API_TRY(c0)
    HIPCHK(hipSetDevice(c0->device));
    Timer t;
    gdr_op_s set;
    set.kind = 2;
    set.ctx = c0;
    set.parts.assign(ops, ops + nops);
    set.n = 0;
    for (int l = 0; l < nops; ++l) set.n = std::max(set.n, ops[l]->n);
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c0->device) ==
                hipSuccess && cus > 0)
            set.list_blocks = 3 * cus;   // the work-list kernel keeps 3 blocks per CU resident
        else
            (void)hipGetLastError();
    }
    const int64_t n = set.n;
    DMem mem;
    double2* b1 = mem.get<double2>((size_t)nops * n);
    double2* x1 = mem.get<double2>((size_t)nops * ns * n);
    // every lattice's first right-hand side, zero beyond its own length
    HIPCHK(hipMemsetAsync(b1, 0, (size_t)nops * n * sizeof(double2), c0->st));
    for (int l = 0; l < nops; ++l) {
        // operators on other contexts: their streams finished their own work
        if (ops[l]->ctx != c0) HIPCHK(hipStreamSynchronize(ops[l]->ctx->st));
        op_pack<double>(ops[l], (const double2*)B[l], b1 + (int64_t)l * n, n, 1, c0->st);
    }
    Stats S(nullptr, (unsigned)p->profile, c0->st, &c0->evpool);
    ManyOut R;
    struct Own {
        ManyOut& r;
        ~Own() {
            for (gdr_defl_s* d : r.defl) delete d;
        }
    } own{R};
    Timer tdr;
    int rc = solve_dr_many(&set, ns, (const double2*)sigma, b1, x1, *p, S, R);
    S.flush();
    HIPCHK(hipStreamSynchronize(c0->st));
    const double t_dr = tdr.sec();
    // ---- per lattice: later right-hand sides, cleanup, final residuals; the
    // lattices of one context in turn, different contexts concurrently
    std::vector<int> rcs(nops, GDR_OK);
    std::vector<std::string> errs(nops);
    std::vector<gdr_ctx_s*> ctxs;
    for (int l = 0; l < nops; ++l)
        if (std::find(ctxs.begin(), ctxs.end(), ops[l]->ctx) == ctxs.end()) ctxs.push_back(ops[l]->ctx);
    auto finish = [&](int l) {
        gdr_op_s* op = ops[l];
        gdr_ctx_s* c = op->ctx;
        gdr_stats* sl = st ? st + l : nullptr;
        try {
            PoolScope ps(c);
            HIPCHK(hipSetDevice(c->device));
            const int64_t nl = op->n;
            DMem lm;
            double2* Beo = lm.get<double2>((size_t)nrhs * nl);
            double2* Xeo = lm.get<double2>((size_t)nrhs * ns * nl);
            op_pack<double>(op, (const double2*)B[l], Beo, nl, nrhs, c->st);
            if (nrhs > 1) check_rhs(op, Beo + nl, nrhs - 1);
            // the first right-hand side's solutions from the batch
            HIPCHK(hipMemcpy2DAsync(Xeo, nl * sizeof(double2), x1 + (int64_t)l * ns * n,
                                    n * sizeof(double2), nl * sizeof(double2), ns,
                                    hipMemcpyDeviceToDevice, c->st));
            Stats Sl(sl, (unsigned)p->profile, c->st, &c->evpool);
            if (sl) {
                sl->cycles_dr = R.cycles[l];
                sl->mvp_dr = R.mvps[l];
                sl->mvp_fp64 = R.cycles[l];
                sl->t_phase[0] = t_dr;
            }
            int r = R.conv[l] ? GDR_OK : GDR_NOT_CONVERGED;
            gdr_defl_s* d = R.defl[l];
            if (nrhs > 1) {
                if (!d) throw GdrError(GDR_ERR_BREAKDOWN, "first solve ended in a lucky breakdown: no deflation space");
                const int r2 = solve_proj_batch(op, d, ns, (const double2*)sigma, nrhs - 1, Beo + nl,
                                                Xeo + (int64_t)ns * nl, 1, *p, Sl);
                if (r2 != GDR_OK) r = r2;
            }
            Timer tc;
            r = cleanup(op, d, ns, (const double2*)sigma, nrhs, Beo, Xeo, *p, Sl);
            if (sl) sl->t_phase[4] += tc.sec();
            Sl.flush();
            r = final_status(r, finish_stats(op, sl, ns, (const double2*)sigma, nrhs, Beo, Xeo, t,
                                             p->precision),
                             p->tol);
            op_unpack<double>(op, Xeo, nl, (double2*)X[l], nrhs * ns, c->st);
            HIPCHK(hipStreamSynchronize(c->st));
            if (sl) sl->t_total = t.sec();
            rcs[l] = r;
        } catch (const GdrError& e) {
            rcs[l] = e.code;
            errs[l] = e.what();
        } catch (const std::bad_alloc&) {
            rcs[l] = GDR_ERR_OOM;
            errs[l] = "device allocation failed";
        } catch (const std::exception& e) {
            rcs[l] = GDR_ERR_HIP;
            errs[l] = e.what();
        }
    };
    {
        std::vector<std::thread> th;
        for (gdr_ctx_s* c : ctxs)
            th.emplace_back([&, c] {
                for (int l = 0; l < nops; ++l)
                    if (ops[l]->ctx == c) finish(l);
            });
        for (auto& x : th) x.join();
    }
    // the batch's own status only says which lattices the first phase left to
    // the cleanup (mixed precision); each lattice's final status decides
    (void)rc;
    int rc_all = GDR_OK;
    for (int l = 0; l < nops; ++l) {
        if (rcs[l] < 0) return fail(c0, rcs[l], errs[l].c_str());
        if (rcs[l] != GDR_OK && rc_all == GDR_OK) rc_all = rcs[l];
    }
    return rc_all;
    API_CATCH(c0)
}

int gdr_defl_k(gdr_defl d) { return d ? d->k : -1; }

int gdr_defl_export(gdr_defl d, gdr_c64* V, gdr_c64* Hbar) {
    if (!d) return GDR_ERR_ARG;
    gdr_op_s* op = d->op;
    gdr_ctx_s* c = op->ctx;
    if (V && !device_ptr(V, c->device))
        return fail(c, GDR_ERR_ARG, "V must be device memory of the context's device");
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    if (V) {
        if (d->prec == GDR_PREC_MIXED)
            op_unpack<float>(op, (const float2*)d->V, op->n, (double2*)V, d->k + 1, c->st);
        else
            op_unpack<double>(op, (const double2*)d->V, op->n, (double2*)V, d->k + 1, c->st);
    }
    if (Hbar && d->k > 0)
        std::memcpy(Hbar, d->Hk_host.data(), d->Hk_host.size() * sizeof(double2));
    HIPCHK(hipStreamSynchronize(c->st));
    return GDR_OK;
    API_CATCH(c)
}

int gdr_defl_import(gdr_op op, int k, const gdr_c64* V, const gdr_c64* Hbar, int precision,
                    gdr_defl* out) {
    if (!op) return GDR_ERR_ARG;
    gdr_ctx_s* c = op->ctx;
    if (!out || !V || (k > 0 && !Hbar) || k < 0 || k > MAXK)
        return fail(c, GDR_ERR_ARG, "bad deflation import arguments");
    if (precision != GDR_PREC_F64 && precision != GDR_PREC_MIXED)
        return fail(c, GDR_ERR_ARG, "precision must be F64 or MIXED");
    *out = nullptr;
    if (!device_ptr(V, c->device))
        return fail(c, GDR_ERR_ARG, "V must be device memory of the context's device");
    for (size_t i = 0; k > 0 && i < (size_t)(k + 1) * k; ++i)
        if (!std::isfinite(Hbar[i].re) || !std::isfinite(Hbar[i].im))
            return fail(c, GDR_ERR_ARG, "Hbar has a non-finite entry");
    gdr_defl_s* d = new gdr_defl_s;
    API_TRY(c)
    HIPCHK(hipSetDevice(c->device));
    d->op = op;
    d->k = k;
    d->prec = precision;
    const int64_t n = op->n;
    if (precision == GDR_PREC_MIXED) {
        const size_t bytes = (size_t)(k + 1 + BASIS_PAD) * n * sizeof(float2);
        HIPCHK(hipMalloc(&d->V, bytes));
        HIPCHK(hipMemsetAsync(d->V, 0, bytes, c->st));
        op_pack<float>(op, (const double2*)V, (float2*)d->V, n, k + 1, c->st);
    } else {
        const size_t bytes = (size_t)(k + 1 + BASIS_PAD) * n * sizeof(double2);
        HIPCHK(hipMalloc(&d->V, bytes));
        HIPCHK(hipMemsetAsync(d->V, 0, bytes, c->st));
        op_pack<double>(op, (const double2*)V, (double2*)d->V, n, k + 1, c->st);
    }
    if (k > 0) {
        d->Hk_host.assign((const double2*)Hbar, (const double2*)Hbar + (size_t)(k + 1) * k);
        HIPCHK(hipMalloc(&d->Hk, (size_t)(k + 1) * k * sizeof(double2)));
        HIPCHK(hipMemcpyAsync(d->Hk, d->Hk_host.data(), d->Hk_host.size() * sizeof(double2),
                              hipMemcpyHostToDevice, c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));
    *out = d;
    return GDR_OK;
    }
    catch (const GdrError& e) {
        delete d;
        return fail(c, e.code, e.what());
    }
}

void gdr_defl_destroy(gdr_defl d) { delete d; }

int gdr_tune_load(const char* path) {
    if (!path) return GDR_ERR_ARG;
    const int k = tune_load(path);
    return k < 0 ? GDR_ERR_ARG : k;
}

int64_t gdr_tune_report(char* buf, int64_t len) {
    const std::string r = tune_report();
    if (buf && len > 0) {
        const size_t k = std::min<size_t>(r.size(), (size_t)(len - 1));
        std::memcpy(buf, r.data(), k);
        buf[k] = 0;
    }
    return (int64_t)r.size();
}

}  // extern "C"
