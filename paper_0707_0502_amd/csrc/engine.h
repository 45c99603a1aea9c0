// Host engine: handles behind the C-ABI and the solver drivers.
#pragma once

#include <list>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <unordered_map>
#include <string>
#include <vector>

#include "gdr.h"
#include "kernels.h"
#include "small.h"

struct GdrError : std::runtime_error {
    int code;
    GdrError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess)                                                             \
            throw GdrError(e_ == hipErrorOutOfMemory ? GDR_ERR_OOM : GDR_ERR_HIP,         \
                           std::string(#x) + ": " + hipGetErrorString(e_));               \
    } while (0)

namespace gdr {
// Device memory cache of a context. Solves allocate their work buffers per
// call; returning them here instead of to the driver lets the next call (or
// the next batch of the same call) reuse them without mapping new memory.
// Best fit within +25 % (sizes rounded up to 2 MiB). The idle blocks of all
// contexts on one device together stay below 60 % of the device's memory:
// returning a block past that releases the returning context's least
// recently returned blocks. An allocation that fails releases the context's
// own idle blocks and retries, then the idle blocks of every other context
// on the device and retries once more. Blocks are only reused in stream
// order on the owning context's stream; hipFree, which releases an idle
// block of another context, waits for the device. Thread safe: one mutex
// per cache, and a registry of the live caches per process.
struct DevPool {
    struct Idle {
        size_t sz;
        void* p;
    };
    std::mutex mu;
    std::list<Idle> lru;   // idle blocks, least recently returned first
    std::multimap<size_t, std::list<Idle>::iterator> bysize;
    std::unordered_map<void*, size_t> used;
    size_t idle_bytes = 0;
    int device = -1;
    // join the registry of `dev` (the device must be current)
    void attach(int dev);
    // leave the registry and release every idle block
    void detach();
    void* get(size_t bytes);   // throws std::bad_alloc
    void put(void* p);
    size_t release();          // idle blocks back to the driver; returns their bytes
    static size_t round(size_t b) {
        const size_t g = b >= (1u << 20) ? (size_t)2 << 20 : (size_t)4 << 10;
        return (b + g - 1) / g * g;
    }

   private:
    void drop_oldest();   // mu held
};
// idle bytes of every cache on `dev`, and their cap
size_t pool_idle_bytes(int dev);
size_t pool_idle_cap(int dev);
}  // namespace gdr

struct gdr_ctx_s {
    int device = 0;
    hipStream_t st = nullptr;    // caller's stream: every result is ordered on it
    hipStream_t aux = nullptr;   // library stream for work that overlaps st
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::string err;
    // timing events of the optional kernel profiler, reused by every solve on
    // this context (creating and destroying thousands per solve costs more
    // than the solve's small kernels)
    std::vector<hipEvent_t> evpool;
    gdr::DevPool pool;
};

struct gdr_op_s {
    gdr_ctx_s* ctx = nullptr;
    gdr::Geom g{};
    int bc[4] = {1, 1, 1, -1};
    double kappa = 0;
    int64_t n = 0;          // 12 * volume
    double2* u64 = nullptr; // FP64 links (internal layout)
    void* ulo = nullptr;    // FP32, FP16, or two-row FP32 (LINK_R12) / FP16 (LINK_R12H) links
    int lst = GDR_LINKS_F32;
    void* ure = nullptr;    // FP16 storage only: FP32 links (lre: FP32 or LINK_R12) for the
    int lre = GDR_LINKS_F32;  //   cleanup's refinement solves
    bool refine = false;    // the FP32 operator reads ure while set (RefineLinks)
    int anti = 0;           // bit mu: direction mu antiperiodic (bc[mu] = -1)
    double su3_dev = -1;    // largest deviation of the links from SU(3) (-1: not checked)
    int kind = 0;             // 0: Wilson-Dirac lattice operator, 1: bidiagonal matrix,
                              // 2: a set of lattices batched together (see parts)
    double2* bd64 = nullptr;  // bidiagonal: diagonal (n) then superdiagonal (n), FP64
    float2* bd32 = nullptr;   //   and the FP32 copy
    // a disc holding the spectrum of A (centre, radius): the s-step basis is
    // built from powers of (A - centre) / radius
    double2 spec_c = {1, 0};
    double spec_r = 1;
    // kind 2: member b of every batched launch is lattice parts[b]; vectors
    // have n = the largest part's n and are zero beyond their own part's n.
    // The FP32 operator of all members runs as one persistent work-list
    // launch of at most list_blocks blocks.
    std::vector<gdr_op_s*> parts;
    int list_blocks = 768;
};

namespace gdr {
// The operator behind a handle: out_v = alpha_v (A - sigma_v) in_v [+ add_v]
// with 1 - sigma_v in dl.d[v] (Wilson: A = I - kappa D; bidiagonal: A = M),
// and the conversions between the caller's canonical complex128 vectors and
// the internal layout of type T.
// mem0: batch member of vector 0 (a set of lattices applies member mem0 + v's
// own operator to vector v; ignored by single operators)
template <typename T>
void op_apply(gdr_op_s* op, const typename CT<T>::t* in, int64_t in_stride,
              typename CT<T>::t* out, int64_t out_stride, const typename CT<T>::t* add,
              int64_t add_stride, const DiagList& dl, int nvec, hipStream_t st,
              const int* act = nullptr, int mem0 = 0);
template <typename T>
void op_pack(gdr_op_s* op, const double2* canon, typename CT<T>::t* dst, int64_t stride, int nvec,
             hipStream_t st);
template <typename T>
void op_unpack(gdr_op_s* op, const typename CT<T>::t* src, int64_t stride, double2* canon, int nvec,
               hipStream_t st);
}  // namespace gdr

namespace gdr {
// Scope in which the FP32 operator of an FP16-storage operator reads its FP32
// link copy (the refinement solves of the mixed-precision cleanup).
struct RefineLinks {
    gdr_op_s* op;
    bool prev;
    explicit RefineLinks(gdr_op_s* o) : op(o), prev(o->refine) { op->refine = op->ure != nullptr; }
    ~RefineLinks() { op->refine = prev; }
};
}  // namespace gdr

struct gdr_defl_s {
    gdr_op_s* op = nullptr;
    int k = 0;
    int prec = GDR_PREC_F64;      // basis storage: F64 (double2) or MIXED (float2)
    void* V = nullptr;            // (k+1) columns of n, internal layout
    double2* Hk = nullptr;        // device (k+1) x k column-major
    std::vector<double2> Hk_host;
    std::vector<double2> extra_sig;   // shift list the extra solutions belong to
    double2* S = nullptr;             // ns x n FP64 (index 0 unused): (A - s_i) S_i = v_{k+1}
    int64_t mvp_extra = 0;
    int cycles_extra = 0;
    ~gdr_defl_s();
};

namespace gdr {

// the memory cache of the context whose API call runs on this thread (set by
// PoolScope at every entry point; one context per host thread)
extern thread_local DevPool* g_pool;
struct PoolScope {
    DevPool* prev;
    explicit PoolScope(gdr_ctx_s* c) : prev(g_pool) { g_pool = c ? &c->pool : nullptr; }
    ~PoolScope() { g_pool = prev; }
};

// device allocation list handed back on scope exit (to the context's cache
// when one is active, else to the driver)
struct DMem {
    std::vector<void*> ptrs;
    DevPool* pool = g_pool;
    ~DMem() {
        for (void* p : ptrs) {
            if (pool)
                pool->put(p);
            else
                (void)hipFree(p);
        }
    }
    template <class X>
    X* get(size_t count) {
        void* p = nullptr;
        if (count == 0) count = 1;
        if (pool) {
            try {
                p = pool->get(count * sizeof(X));
            } catch (const std::bad_alloc&) {
                throw GdrError(GDR_ERR_OOM, "device allocation failed");
            }
        } else {
            HIPCHK(hipMalloc(&p, count * sizeof(X)));
        }
        ptrs.push_back(p);
        return (X*)p;
    }
};

// Optional HIP-event timing of kernel classes (bitmask), on the context
// stream, with the algorithmic bytes and flops of every timed launch.
struct Prof {
    unsigned mask = 0;
    hipStream_t st = nullptr;
    struct Rec {
        int cls;
        double bytes, flops;
        hipEvent_t a, b;
    };
    std::vector<Rec> pend;
    std::vector<hipEvent_t> own;
    std::vector<hipEvent_t>* pool = &own;   // the context's pool when one is given
    hipEvent_t cur = nullptr;
    double ms[8] = {}, bytes[8] = {}, flops[8] = {};
    int64_t cnt[8] = {};
    bool on(int cls) const { return (mask >> cls) & 1u; }
    hipEvent_t get() {
        hipEvent_t e;
        if (!pool->empty()) {
            e = pool->back();
            pool->pop_back();
        } else {
            HIPCHK(hipEventCreate(&e));
        }
        return e;
    }
    void begin(int cls) {
        if (!on(cls)) return;
        cur = get();
        HIPCHK(hipEventRecord(cur, st));
    }
    void end(int cls, double b, double f) {
        if (!on(cls)) return;
        hipEvent_t e = get();
        HIPCHK(hipEventRecord(e, st));
        pend.push_back({cls, b, f, cur, e});
        if (pend.size() > 2048) harvest();
    }
    // interval on another stream: mark() before the work, span() after it
    hipEvent_t mark(int cls, hipStream_t s) {
        if (!on(cls)) return nullptr;
        hipEvent_t e = get();
        HIPCHK(hipEventRecord(e, s));
        return e;
    }
    void span(int cls, hipEvent_t a, hipStream_t s, double b, double f) {
        if (!on(cls) || !a) return;
        hipEvent_t e = get();
        HIPCHK(hipEventRecord(e, s));
        pend.push_back({cls, b, f, a, e});
    }
    void harvest() {
        if (pend.empty()) return;
        for (auto& r : pend) HIPCHK(hipEventSynchronize(r.b));
        for (auto& r : pend) {
            float t = 0;
            HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
            ms[r.cls] += t;
            bytes[r.cls] += r.bytes;
            flops[r.cls] += r.flops;
            cnt[r.cls] += 1;
            pool->push_back(r.a);
            pool->push_back(r.b);
        }
        pend.clear();
    }
    ~Prof() {
        for (auto& r : pend) {
            pool->push_back(r.a);
            pool->push_back(r.b);
        }
        for (hipEvent_t e : own) (void)hipEventDestroy(e);
    }
};

struct Stats {
    gdr_stats* st = nullptr;
    Prof prof;
    Stats(gdr_stats* s, unsigned mask, hipStream_t stream,
          std::vector<hipEvent_t>* evpool = nullptr)
        : st(s) {
        prof.mask = mask;
        prof.st = stream;
        if (evpool) prof.pool = evpool;
    }
    void flush() {
        prof.harvest();
        if (!st) return;
        for (int c = 0; c < 8; ++c) {
            st->k_ms[c] += prof.ms[c];
            st->k_bytes[c] += prof.bytes[c];
            st->k_flops[c] += prof.flops[c];
            st->k_launches[c] += prof.cnt[c];
            prof.ms[c] = prof.bytes[c] = prof.flops[c] = 0;
            prof.cnt[c] = 0;
        }
    }
    void hist(int phase, int cycle, int64_t mvps, double r1, double rmax) {
        if (!st || !st->hist || st->hist_len >= st->hist_cap) return;
        double* h = st->hist + 5 * st->hist_len++;
        h[0] = phase;
        h[1] = cycle;
        h[2] = (double)mvps;
        h[3] = r1;
        h[4] = rmax;
    }
    void theta(const double2* t, int k) {
        if (!st || !st->theta) return;
        for (int i = 0; i < k && st->theta_len < st->theta_cap; ++i)
            st->theta[st->theta_len++] = gdr_c64{t[i].x, t[i].y};
    }
};

// GMRES-DR-Sh on the first right-hand sides of a set of lattices (op->kind
// == 2) as one batch, mixed precision: member b's right-hand side at
// b_eo + b*n, its solutions at X + b*ns*n (n = op->n); per-member results and
// deflation pairs (each for its own lattice, owned by the caller) in R.
struct ManyOut {
    std::vector<int> conv, cycles;
    std::vector<int64_t> mvps;
    std::vector<gdr_defl_s*> defl;
};
int solve_dr_many(gdr_op_s* op, int ns, const double2* sig, const double2* b_eo, double2* X,
                  const gdr_params& p, Stats& S, ManyOut& R);

// whole-problem solver (internal layouts); returns GDR_OK / GDR_NOT_CONVERGED
int solve_dr_sh(gdr_op_s* op, int ns, const double2* sig, const double2* b_eo, double2* X_eo,
                const gdr_params& p, Stats& S, gdr_defl_s** defl_out, bool* converged);
// nprev: right-hand sides (and their solutions) already solved, stored just
// before B_eo and X_eo, used by the related right-hand side projection
int solve_proj_batch(gdr_op_s* op, gdr_defl_s* defl, int ns, const double2* sig, int nrhs,
                     const double2* B_eo, double2* X_eo, int nprev, const gdr_params& p, Stats& S);
// true FP64 residual norms ||b_j - (A - s_i) x_ij|| / ||b_j||, resid[j*ns + i]
void true_residuals(gdr_op_s* op, int ns, const double2* sig, int nrhs, const double2* B_eo,
                    const double2* X_eo, std::vector<double>& resid);
// mixed-precision cleanup: FP64-refined single-shift GMRES(m)-Proj(k) per (shift, RHS)
int cleanup(gdr_op_s* op, gdr_defl_s* defl, int ns, const double2* sig, int nrhs,
            const double2* B_eo, double2* X_eo, const gdr_params& p, Stats& S);
// device address of gdr_op_apply_noalloc's static workspace on `device`,
// looked up once per device (the device must be current); GDR_OK or GDR_ERR_HIP
int noalloc_setup(int device);
// true if p is device (or managed) memory usable on `device`
bool device_ptr(const void* p, int device);
double vec_norm(gdr_op_s* op, const double2* x);
// 2-norms of nv FP64 vectors stored n apart
std::vector<double> norms_of(gdr_op_s* op, const double2* X, int nv);

}  // namespace gdr
