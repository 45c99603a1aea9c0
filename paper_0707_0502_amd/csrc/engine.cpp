// Solver drivers: GMRES-DR-Sh (or FOM-DR-Sh) for the first right-hand side (Sec. 3), the
// batched GMRES-Proj-Sh phase for the extra right-hand side v_{k+1} and the
// later right-hand sides with the correction (Sec. 4), and the FP64-refined
// cleanup of the mixed-precision path.
//
// Host code only orders kernels on the context stream and reads back one
// small record per restart cycle (the shortcut residual norm, the new
// beta_i, flags and the kept harmonic Ritz values).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>

#include "engine.h"
#include "tune.h"

gdr_defl_s::~gdr_defl_s() {
    if (V) (void)hipFree(V);
    if (Hk) (void)hipFree(Hk);
    if (S) (void)hipFree(S);
}

namespace gdr {

static inline double2 z(double r, double i = 0) { return make_double2(r, i); }

thread_local DevPool* g_pool = nullptr;
static inline double zabs(double2 a) { return std::hypot(a.x, a.y); }

template <typename T>
static const void* links_for(gdr_op_s* op) {
    return std::is_same<T, double>::value ? (const void*)op->u64 : op->refine ? op->ure : op->ulo;
}
template <typename T>
static int lst_for(gdr_op_s* op) {
    return std::is_same<T, double>::value ? GDR_LINKS_F64 : op->refine ? op->lre : op->lst;
}

// algorithmic bytes of one Wilson launch over nvec vectors: every link and
// every spinor component once (links shared by the vectors of one launch)
template <typename T>
static double dslash_bytes(gdr_op_s* op, int nvec, bool add) {
    double cs = std::is_same<T, double>::value ? 16 : 8;
    if (op->kind == 2) {   // a set of lattices: the mean member's bytes per vector
        double b = 0;
        for (gdr_op_s* q : op->parts) b += dslash_bytes<T>(q, 1, add);
        return op->parts.empty() ? 0 : b * nvec / op->parts.size();
    }
    if (op->kind == 1)   // bidiagonal: 2n matrix entries, in, out (, add) per vector
        return (double)op->n * cs * (2 + nvec * (2 + (add ? 1 : 0)));
    const double vol = op->g.vol;
    const int ls = lst_for<T>(op);
    double link = std::is_same<T, double>::value ? 16 * 36
                  : ls == LINK_R12              ? 8 * 24
                  : ls == LINK_R12H             ? 4 * 24
                  : ls == GDR_LINKS_F16         ? 4 * 36
                                                : 8 * 36;
    return vol * (link + nvec * (12 * cs * 2 + (add ? 12 * cs : 0)));
}
static double dslash_flops(gdr_op_s* op, int nvec) {
    if (op->kind == 2) {
        double f = 0;
        for (gdr_op_s* q : op->parts) f += dslash_flops(q, 1);
        return op->parts.empty() ? 0 : f * nvec / op->parts.size();
    }
    if (op->kind == 1) return (double)op->n * nvec * 16.0;
    return (double)op->g.vol * nvec * 1368.0;
}

template <typename T>
void op_apply(gdr_op_s* op, const typename CT<T>::t* in, int64_t in_stride,
              typename CT<T>::t* out, int64_t out_stride, const typename CT<T>::t* add,
              int64_t add_stride, const DiagList& dl, int nvec, hipStream_t st, const int* act,
              int mem0) {
    if (op->kind == 2) {
        if (nvec < 1) return;
        if (mem0 < 0 || mem0 + nvec > (int)op->parts.size())
            throw std::invalid_argument("lattice set: members out of range");
        if constexpr (std::is_same<T, float>::value) {
            // every member's operator in one persistent work-list launch
            if (add) throw std::invalid_argument("lattice set: FP32 launches add no vector");
            LatList L{};
            L.nm = nvec;
            int ls = -1;
            for (int v = 0; v < nvec; ++v) {
                gdr_op_s* q = op->parts[mem0 + v];
                L.g[v] = q->g;
                L.links[v] = links_for<T>(q);
                L.kappa[v] = (float)q->kappa;
                L.anti[v] = q->anti;
                L.tile0[v + 1] = L.tile0[v] + (int)(q->g.vol >> 8);
                const int lq = lst_for<T>(q);
                if (ls >= 0 && lq != ls) throw std::invalid_argument("lattice set: mixed link storage");
                ls = lq;
            }
            dslash_list(in, in_stride, out, out_stride, L, ls, dl, st, act, op->list_blocks);
        } else {
            // FP64: each member on its own lattice (once per restart cycle)
            for (int v = 0; v < nvec; ++v) {
                DiagList d1{};
                d1.d[0] = dl.d[v];
                d1.alpha[0] = dl.alpha[v];
                op_apply<T>(op->parts[mem0 + v], in + v * in_stride, in_stride, out + v * out_stride,
                            out_stride, add ? add + v * add_stride : nullptr, add_stride, d1, 1, st,
                            act ? act + v : nullptr);
            }
        }
        return;
    }
    if (op->kind == 1) {
        const typename CT<T>::t* de;
        if constexpr (std::is_same<T, double>::value) de = op->bd64;
        else de = op->bd32;
        bidiag_apply<T>(in, in_stride, out, out_stride, add, add_stride, de, op->n, dl, nvec, st,
                        act);
        return;
    }
    dslash<T>(in, in_stride, out, out_stride, add, add_stride, links_for<T>(op), lst_for<T>(op),
              op->g, op->kappa, dl, nvec, st, act, op->anti);
}
template <typename T>
void op_pack(gdr_op_s* op, const double2* canon, typename CT<T>::t* dst, int64_t stride, int nvec,
             hipStream_t st) {
    if (op->kind == 1) plain_copy<double, T>(canon, op->n, dst, stride, op->n, nvec, st);
    else pack_spinor<T>(canon, dst, stride, op->g, nvec, st);
}
template <typename T>
void op_unpack(gdr_op_s* op, const typename CT<T>::t* src, int64_t stride, double2* canon, int nvec,
               hipStream_t st) {
    if (op->kind == 1) plain_copy<T, double>(src, stride, canon, op->n, op->n, nvec, st);
    else unpack_spinor<T>(src, stride, canon, op->g, nvec, st);
}
template void op_apply<double>(gdr_op_s*, const double2*, int64_t, double2*, int64_t,
                               const double2*, int64_t, const DiagList&, int, hipStream_t,
                               const int*, int);
template void op_apply<float>(gdr_op_s*, const float2*, int64_t, float2*, int64_t, const float2*,
                              int64_t, const DiagList&, int, hipStream_t, const int*, int);
template void op_pack<double>(gdr_op_s*, const double2*, double2*, int64_t, int, hipStream_t);
template void op_pack<float>(gdr_op_s*, const double2*, float2*, int64_t, int, hipStream_t);
template void op_unpack<double>(gdr_op_s*, const double2*, int64_t, double2*, int, hipStream_t);
template void op_unpack<float>(gdr_op_s*, const float2*, int64_t, double2*, int, hipStream_t);

// Krylov bases carry BASIS_PAD zeroed spare columns: the Gram-Schmidt
// kernels load columns in chunks of 8 without per-column guards.
template <typename T>
static typename CT<T>::t* alloc_basis(DMem& mem, int cols, int64_t n, hipStream_t st) {
    using C = typename CT<T>::t;
    const size_t cnt = (size_t)(cols + BASIS_PAD) * n;
    C* p = mem.get<C>(cnt);
    HIPCHK(hipMemsetAsync(p, 0, cnt * sizeof(C), st));
    return p;
}

double vec_norm(gdr_op_s* op, const double2* x) {
    DMem mem;
    hipStream_t st = op->ctx->st;
    const int nblk = cgs_nblk(op->n);
    double2* part = mem.get<double2>(nblk);
    double2* out = mem.get<double2>(1);
    gs_dot<double, double>(nullptr, 0, 0, 0, x, 0, nullptr, 0, part, nblk, op->n, 1, st);
    reduce_cols(part, nblk, 1, out, 1, nullptr, 0, 1, st);
    double2 h;
    HIPCHK(hipMemcpyAsync(&h, out, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return std::sqrt(h.x);
}

// ---------------------------------------------------------------------------
// Batched Arnoldi step (eq. (2.2)) with CGS2: one operator launch and three
// sweeps over each member's basis per step.
// Arnoldi recurrence (eq. (2.2)) with delayed classical Gram-Schmidt
// (DCGS2): the operator is applied to the once-orthogonalised candidate r_j in
// column j, and one projection sweep V_{0..j}^H [r_j, A r_j] plus one update
// sweep both finish column j (its second Gram-Schmidt pass, folded into the
// correction of H column j-1) and produce the next candidate r_{j+1} in
// column j+1. In exact arithmetic this is the same basis and Hessenberg
// matrix as CGS2 (orthogonalise twice); the last candidate is finished by
// close(). Two sweeps over the basis per step instead of three.
template <typename T>
struct Arnoldi {
    using C = typename CT<T>::t;
    gdr_op_s* op = nullptr;
    hipStream_t st = nullptr;
    int m = 0, nmem = 0;
    int64_t n = 0;
    C* V = nullptr;
    int64_t vms = 0;
    C* w = nullptr;
    double2* H = nullptr;
    int64_t hms = 0;
    double* inv = nullptr;
    int* brk = nullptr;
    double2* partial = nullptr;
    int nblk = 0;
    double2* G = nullptr;       // reduced projection sums, GMS per member
    double2* coef = nullptr;    // update coefficients, GS_COEF_MS per member
    double* ref = nullptr;      // ||A q_{j-1}|| estimate per member (breakdown test)
    static constexpr int GMS = 2 * (MAXM + 1) + 2;
    DiagList dl{};
    Prof* prof = nullptr;
    // s-step cycle (FP32 only): block size, reduced block sums, P1, raw norms,
    // block coefficients, and the scaled shifted operator of the powers
    int sblk = 0;
    static constexpr int BGS = BLK_MAX * (MAXM + 1 + BLK_MAX);
    double2* Gb = nullptr;
    double2* Psave = nullptr;
    double* znorm = nullptr;
    double2* bcoef = nullptr;
    int* reo = nullptr;         // per member: the block needs its second sweep pair
    double reorth = 20;
    DiagList dlp{};

    void init(DMem& mem, gdr_op_s* op_, int m_, int nmem_, C* Vbuf, int64_t vms_) {
        op = op_;
        st = op->ctx->st;
        m = m_;
        nmem = nmem_;
        n = op->n;
        V = Vbuf;
        vms = vms_;
        w = mem.get<C>(n * nmem);
        hms = (int64_t)(m + 1) * m;
        H = mem.get<double2>(hms * nmem);
        inv = mem.get<double>(nmem);
        brk = mem.get<int>(nmem);
        nblk = cgs_nblk(n, nmem, std::is_same<T, float>::value);
        partial = mem.get<double2>((size_t)std::max({80, 2 * m + 4, BLK_MAX * (m + 1 + BLK_MAX)}) *
                                   nblk * nmem);
        Gb = mem.get<double2>((size_t)BGS * nmem);
        Psave = mem.get<double2>((size_t)(MAXM + 1) * BLK_MAX * nmem);
        znorm = mem.get<double>((size_t)BLK_MAX * nmem);
        bcoef = mem.get<double2>((size_t)BLK_COEF_MS * nmem);
        reo = mem.get<int>(nmem);
        G = mem.get<double2>((size_t)GMS * nmem);
        coef = mem.get<double2>((size_t)GS_COEF_MS * nmem);
        ref = mem.get<double>(nmem);
        for (int v = 0; v < DSLASH_MAXV; ++v) {
            dl.d[v] = z(1);
            dl.alpha[v] = 1;
            // (A - c) / r: the operator's diagonal factor 1 - c, scale 1 / r
            // (a set of lattices: each member's own disc)
            const gdr_op_s* q = op->kind == 2 && v < (int)op->parts.size() ? op->parts[v] : op;
            dlp.d[v] = z(1.0 - q->spec_c.x, -q->spec_c.y);
            dlp.alpha[v] = 1.0 / q->spec_r;
        }
        if (op->kind == 2) {
            if (nmem != (int)op->parts.size() || nmem > DSLASH_MAXV)
                throw std::invalid_argument("lattice set: one batch member per lattice, at most 16");
            std::vector<double2> th(nmem);
            std::vector<double> rh(nmem);
            for (int b = 0; b < nmem; ++b) {
                th[b] = op->parts[b]->spec_c;
                rh[b] = op->parts[b]->spec_r;
            }
            thetas = mem.get<double2>(nmem);
            rhos = mem.get<double>(nmem);
            HIPCHK(hipMemcpyAsync(thetas, th.data(), nmem * sizeof(double2), hipMemcpyHostToDevice, st));
            HIPCHK(hipMemcpyAsync(rhos, rh.data(), nmem * sizeof(double), hipMemcpyHostToDevice, st));
        }
    }
    double2* thetas = nullptr;   // lattice sets: per-member disc of the s-step powers
    double* rhos = nullptr;

    // Block size of the cycle: s-step blocks only for the FP32 basis
    void set_block(int s, double reorth_ = 20) {
        sblk = (std::is_same<T, float>::value && s >= 2) ? std::min(s, BLK_MAX) : 0;
        // blocks of more than 4 run on the matrix-core sweeps, in 16-row chunks
        if (sblk > 4 && n % 16 != 0) sblk = 4;
        reorth = reorth_;
    }

    // s-step cycle: from the orthonormal column j, sb = min(sblk, m - j) powers
    // z_i = (A - c) z_{i-1} / r go straight into columns j+1..j+sb. One block
    // projection sweep against columns 0..j (its basis range also takes in the
    // block, giving the block's Gram matrix), the Cholesky factor of the
    // Gram matrix with the projection removed, and one update sweep give the
    // new orthonormal columns; a member whose projection cancelled more than
    // the reorth ratio of a block vector takes a second projection and update
    // sweep (kernels masked by reo). H columns j..j+sb-1 follow from the
    // change of basis (sstep_small). Two sweeps over the basis per block of
    // sb steps, four with the second pair.
    void blocks(int j0, const int* act, int nact) {
        const double cs = sizeof(C);
        const double dn = (double)n * nact;
        for (int j = j0; j < m;) {
            const int sb = std::min(sblk, m - j);
            C* Z = V + (int64_t)(j + 1) * n;
            for (int i = 1; i <= sb; ++i) {
                const C* src = V + (int64_t)(j + i - 1) * n;
                C* dst = V + (int64_t)(j + i) * n;
                for (int b0 = 0; b0 < nmem; b0 += DSLASH_MAXV) {
                    const int nb = std::min(DSLASH_MAXV, nmem - b0);
                    prof->begin(GDR_K_DSLASH);
                    op_apply<T>(op, src + b0 * vms, vms, dst + b0 * vms, vms, nullptr, 0, dlp, nb, st,
                                act ? act + b0 : nullptr, b0);
                    const int na = std::min(nb, nact - std::min(nact, b0));
                    prof->end(GDR_K_DSLASH, dslash_bytes<T>(op, na, false), dslash_flops(op, na));
                }
            }
            const int nc = j + 1 + sb;
            SstepArgs sa{};
            sa.G = Gb;
            sa.g_ms = BGS;
            sa.j = j;
            sa.sb = sb;
            sa.m = m;
            sa.Psave = Psave;
            sa.p_ms = (int64_t)(MAXM + 1) * BLK_MAX;
            sa.znorm = znorm;
            sa.coef = bcoef;
            sa.coef_ms = BLK_COEF_MS;
            sa.H = H;
            sa.ldh = m + 1;
            sa.h_ms = hms;
            sa.theta = op->spec_c;
            sa.rho = op->spec_r;
            sa.thetas = thetas;
            sa.rhos = rhos;
            sa.brk = brk;
            sa.reorth = reorth;
            fill_int(reo, 0, nmem, st);
            for (int pass = 1; pass <= 2; ++pass) {
                // the second pair only for the members mode 1 flagged; which
                // ones is decided on the device, so its launches are timed in
                // their own class without algorithmic bytes
                const bool second = pass == 2;
                const int* msk = second ? reo : act;
                const int kp = second ? GDR_K_GS_CLOSE : GDR_K_GS_PROJECT;
                const int ku = second ? GDR_K_GS_CLOSE : GDR_K_GS_UPDATE;
                prof->begin(kp);
                blk_dot<T>(V, n, vms, nc, Z, n, vms, sb, partial, nblk, n, nmem, st, msk, second);
                // algorithmic bytes: columns 0..j and the block once each (the
                // sweep reads the block twice, as basis columns and as inputs)
                prof->end(kp, second ? 0.0 : dn * nc * cs, second ? 0.0 : dn * 16.0 * nc * sb);
                reduce_cols(partial, nblk, sb * nc, Gb, BGS, nullptr, 0, nmem, st, msk);
                sa.mode = pass;
                sa.act = msk;
                sa.reo = second ? nullptr : reo;
                sstep_small(sa, nmem, st);
                prof->begin(ku);
                blk_update<T>(V, n, vms, j + 1, Z, n, vms, sb, bcoef, BLK_COEF_MS, n, nmem, st, msk,
                              second);
                prof->end(ku, second ? 0.0 : dn * (j + 1 + 2.0 * sb) * cs,
                          second ? 0.0 : dn * 16.0 * (j + 1 + sb) * sb);
            }
            j += sb;
        }
    }

    // Step j: column j holds the candidate r_j (columns 0..j-1 final); j0 is
    // the first step of the cycle (column j0 already orthonormal, H columns
    // before it final).
    void step(int j, int j0, const int* act, int nact) {
        const double cs = sizeof(C);
        const double dn = (double)n * nact;
        C* col = V + (int64_t)j * n;
        for (int b0 = 0; b0 < nmem; b0 += DSLASH_MAXV) {
            const int nb = std::min(DSLASH_MAXV, nmem - b0);
            prof->begin(GDR_K_DSLASH);
            op_apply<T>(op, col + b0 * vms, vms, w + b0 * n, n, nullptr, 0, dl, nb, st,
                        act ? act + b0 : nullptr, b0);
            const int na = std::min(nb, nact - std::min(nact, b0));
            prof->end(GDR_K_DSLASH, dslash_bytes<T>(op, na, false), dslash_flops(op, na));
        }
        const double nc = j + 1;
        prof->begin(GDR_K_GS_PROJECT);
        gs_dot<T, T>(V, n, vms, j + 1, col, vms, w, n, partial, nblk, n, nmem, st, act);
        prof->end(GDR_K_GS_PROJECT, dn * (nc + 1) * cs, dn * 16 * (nc + 1));
        reduce_cols(partial, nblk, 2 * (j + 1) + 1, G, GMS, nullptr, 0, nmem, st, act);
        dcgs_coef(G, GMS, j, 2, j == j0, H, m + 1, hms, coef, GS_COEF_MS, ref, brk, 1e-14, nmem,
                  st, act);
        prof->begin(GDR_K_GS_UPDATE);
        gs_update<T>(V, n, vms, j, col, vms, w, n, col, vms, col + n, vms, coef, GS_COEF_MS, n,
                     nmem, st, act);
        prof->end(GDR_K_GS_UPDATE, dn * (j + 4) * cs, dn * 16 * j);
    }

    // One Arnoldi cycle: steps j0..m-1 and the closing pass, breakdown flags
    // reset first. With `graph`, the cycle is captured once per (basis, H,
    // j0) into a HIP graph and replayed (every argument of these launches is
    // fixed; the per-member active flags are read from device memory).
    struct Cached {
        const void* v;
        const void* h;
        int j0;
        hipGraph_t g;
        hipGraphExec_t e;
    };
    std::vector<Cached> graphs;
    bool use_graph = false;
    int eager_tuning = 0;   // cycles run eagerly for the launch tuner

    void body(int j0, const int* act, int nact) {
        fill_int(brk, -1, nmem, st);
        if constexpr (std::is_same<T, float>::value) {
            if (sblk >= 2) {
                blocks(j0, act, nact);
                return;
            }
        }
        for (int j = j0; j < m; ++j) step(j, j0, act, nact);
        close(act, nact);
    }

    void cycle(int j0, const int* act, int nact) {
        // the legacy null stream cannot be captured: eager launches there
        if (!use_graph || prof->mask || st == nullptr) {
            body(j0, act, nact);
            return;
        }
        // while the launch tuner still times this cycle's kernels, the cycle
        // runs eagerly (captured launches are not timed); at most 4 such cycles
        if (eager_tuning < 4 && tune_active()) {
            const long before = tune_new_open();
            body(j0, act, nact);
            ++eager_tuning;
            if (tune_new_open() == before && tune_open() == 0) eager_tuning = 4;
            return;
        }
        for (auto& c : graphs)
            if (c.v == V && c.h == H && c.j0 == j0) {
                HIPCHK(hipGraphLaunch(c.e, st));
                return;
            }
        Cached c{V, H, j0, nullptr, nullptr};
        {
            TuneCaptureGuard quiet;   // no tuner event calls in any thread meanwhile
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            body(j0, act, nact);
            HIPCHK(hipStreamEndCapture(st, &c.g));
        }
        HIPCHK(hipGraphInstantiate(&c.e, c.g, nullptr, nullptr, 0));
        graphs.push_back(c);
        HIPCHK(hipGraphLaunch(c.e, st));
    }

    ~Arnoldi() {
        for (auto& c : graphs) {
            if (c.e) (void)hipGraphExecDestroy(c.e);
            if (c.g) (void)hipGraphDestroy(c.g);
        }
    }

    // Finish the last candidate (column m): second pass against columns 0..m-1.
    void close(const int* act, int nact) {
        const double cs = sizeof(C);
        const double dn = (double)n * nact;
        C* col = V + (int64_t)m * n;
        prof->begin(GDR_K_GS_CLOSE);
        gs_dot<T, T>(V, n, vms, m + 1, col, vms, (const C*)nullptr, 0, partial, nblk, n, nmem, st,
                     act);
        reduce_cols(partial, nblk, m + 2, G, GMS, nullptr, 0, nmem, st, act);
        dcgs_coef(G, GMS, m, 1, 0, H, m + 1, hms, coef, GS_COEF_MS, ref, brk, 1e-14, nmem, st, act);
        gs_update<T>(V, n, vms, m, col, vms, (const C*)nullptr, 0, col, vms, (C*)nullptr, 0, coef,
                     GS_COEF_MS, n, nmem, st, act);
        prof->end(GDR_K_GS_CLOSE, dn * (2.0 * (m + 1) + 1) * cs, dn * 16.0 * m);
    }
};

// Orthonormalise column k of Vb against columns 0..k-1 in place: classical
// Gram-Schmidt twice, each pass one projection sweep and one update sweep.
template <typename T>
static void orth_column(gdr_op_s* op, typename CT<T>::t* Vb, int k, double2* partial, int nblk,
                        double2* tG, double2* tcoef, double* tref, int* tbrk) {
    using C = typename CT<T>::t;
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    C* col = Vb + (int64_t)k * n;
    for (int pass = 0; pass < 2; ++pass) {
        fill_int(tbrk, -1, 1, st);
        gs_dot<T, T>(Vb, n, 0, k + 1, col, 0, (const C*)nullptr, 0, partial, nblk, n, 1, st);
        reduce_cols(partial, nblk, k + 2, tG, 0, nullptr, 0, 1, st);
        dcgs_coef(tG, 0, k, 1, 1, nullptr, 0, 0, tcoef, 0, tref, tbrk, 0.0, 1, st);
        gs_update<T>(Vb, n, 0, k, col, 0, (const C*)nullptr, 0, col, 0, (C*)nullptr, 0, tcoef, 0, n,
                     1, st);
    }
}

// ---------------------------------------------------------------------------
// GMRES-DR(m,k)-Sh on one right-hand side (algorithm GMRES-DR-Sh, Sec. 3)
template <typename T>
static int dr_run(gdr_op_s* op, int ns, const double2* sig_h, const double2* b_eo, double2* X,
                  const gdr_params& p, Stats& S, gdr_defl_s** defl_out, bool* conv_out) {
    using C = typename CT<T>::t;
    constexpr bool mixed = std::is_same<T, float>::value;
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    const int m = p.m_dr, k = p.k;
    DMem mem;
    C* Va = alloc_basis<T>(mem, m + 1, n, st);
    C* Vb = alloc_basis<T>(mem, m + 1, n, st);
    Arnoldi<T> A;
    A.init(mem, op, m, 1, Va, 0);
    A.use_graph = p.use_graph != 0;
    A.set_block(p.sstep, p.sstep_reorth);
    A.prof = &S.prof;
    double2* Hn = mem.get<double2>((size_t)(m + 1) * m);
    double2* c0 = mem.get<double2>(m + 1);
    double2* c1 = mem.get<double2>(m + 1);
    double2* coef = mem.get<double2>((size_t)(m + 1) * (ns + 1));
    double2* P = mem.get<double2>((size_t)(m + 1) * (k + 1));
    CycleOut* outs = mem.get<CycleOut>(2);
    double2* sig = mem.get<double2>(ns);
    double2* tH = mem.get<double2>(256);
    double2* tcoef = mem.get<double2>(GS_COEF_MS);
    double* tinv = mem.get<double>(2);
    int* tbrk = mem.get<int>(2);
    double* dsc = mem.get<double>(2);
    double2* rtrue = mixed ? mem.get<double2>(n) : nullptr;
    HIPCHK(hipMemcpyAsync(sig, sig_h, ns * sizeof(double2), hipMemcpyHostToDevice, st));

    const double bnorm = vec_norm(op, b_eo);
    if (!std::isfinite(bnorm)) throw GdrError(GDR_ERR_ARG, "right-hand side is not finite");
    HIPCHK(hipMemsetAsync(X, 0, (size_t)ns * n * sizeof(double2), st));
    if (!(bnorm > 0)) {
        *conv_out = true;
        if (defl_out) *defl_out = nullptr;
        HIPCHK(hipStreamSynchronize(st));
        return GDR_OK;
    }
    CycleOut init{};
    init.snorm = bnorm;
    for (int i = 0; i < MAXNS; ++i) init.beta[i] = z(1);
    HIPCHK(hipMemcpyAsync(&outs[0], &init, sizeof(CycleOut), hipMemcpyHostToDevice, st));
    std::vector<double2> ch(m + 1, z(0));
    ch[0] = z(bnorm);
    HIPCHK(hipMemcpyAsync(c0, ch.data(), (m + 1) * sizeof(double2), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(Hn, 0, (size_t)(m + 1) * m * sizeof(double2), st));
    HIPCHK(hipMemsetAsync(A.H, 0, (size_t)(m + 1) * m * sizeof(double2), st));
    const double invb = 1.0 / bnorm;
    HIPCHK(hipMemcpyAsync(dsc, &invb, sizeof(double), hipMemcpyHostToDevice, st));
    convert_scale<T>(b_eo, 0, dsc, 0, Va, 0, n, 1, st);

    int cur = 1, prv = 0;
    C* Vc = Va;
    C* Vn = Vb;
    double2* Hc = A.H;
    double2* Hx = Hn;
    double2* cc = c0;
    double2* cx = c1;
    int j0 = 0, cycles = 0, brk = -1;
    int64_t mvps = 0;
    bool conv = false;
    double best_true = std::numeric_limits<double>::infinity();
    int stall = 0;
    const unsigned allx = ns >= 32 ? 0xffffffffu : ((1u << ns) - 1u);
    for (int cyc = 0; cyc < p.max_cycles; ++cyc) {
        ++cycles;
        A.V = Vc;
        A.H = Hc;
        A.cycle(j0, nullptr, 1);
        mvps += m - j0;
        HIPCHK(hipMemsetAsync(&outs[cur].flags, 0, sizeof(int), st));
        CycleArgs a{};
        a.H = Hc;
        a.c = cc;
        a.sigma = sig;
        a.beta = outs[prv].beta;
        a.brk = A.brk;
        a.coef = coef;
        a.out = &outs[cur];
        a.restart = 0;
        a.k = k;
        a.P = P;
        a.Hnew = Hx;
        a.cnew = cx;
        a.m = m;
        a.ns = ns;
        a.galerkin = p.galerkin;
        S.prof.begin(GDR_K_SMALL);
        cycle_small(a, 1, st);
        S.prof.end(GDR_K_SMALL, 0, 0);
        // the restart half (harmonic Ritz, Schur form, P, new H and c) runs on
        // the auxiliary stream while the solution update and the FP64 residual
        // run here; nothing below reads its outputs before the join
        gdr_ctx_s* cx_ = op->ctx;
        HIPCHK(hipEventRecord(cx_->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(cx_->aux, cx_->ev_fork, 0));
        {
            CycleArgs ar = a;
            ar.restart = 2;
            hipEvent_t pm = S.prof.mark(GDR_K_SMALL, cx_->aux);
            cycle_small(ar, 1, cx_->aux);
            S.prof.span(GDR_K_SMALL, pm, cx_->aux, 0, 0);
        }
        HIPCHK(hipEventRecord(cx_->ev_join, cx_->aux));
        S.prof.begin(GDR_K_COMBINE);
        vcombine<T>(Vc, n, 0, m, coef, m + 1, 0, ns, X, n, 0, allx, n, 1, st);
        S.prof.end(GDR_K_COMBINE, (double)n * (m * sizeof(C) + 32.0 * ns), (double)n * m * ns * 8);
        double rtn = 0;
        if (mixed) {
            DiagList dl{};
            dl.d[0] = z(1.0 - sig_h[0].x, -sig_h[0].y);
            dl.alpha[0] = -1;
            // FP64 true residual: its own class (the operator class holds the
            // FP32 operator of the Krylov space only)
            S.prof.begin(GDR_K_OTHER);
            op_apply<double>(op, X, 0, rtrue, 0, b_eo, 0, dl, 1,
                           st);
            S.prof.end(GDR_K_OTHER, dslash_bytes<double>(op, 1, true), dslash_flops(op, 1));
            if (S.st) S.st->mvp_fp64 += 1;
        }
        HIPCHK(hipStreamWaitEvent(st, cx_->ev_join, 0));
        CycleOut o;
        HIPCHK(hipMemcpyAsync(&o, &outs[cur], sizeof(CycleOut), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(&brk, A.brk, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (mixed) rtn = vec_norm(op, rtrue);
        if (o.flags & 1)
            throw GdrError(GDR_ERR_BREAKDOWN, p.galerkin ? "FOM-DR-Sh: singular Galerkin system (H_m - sigma_i I)"
                                                         : "GMRES-DR-Sh: singular shifted system ((Q^H s)_{m+1} = 0)");
        if (o.flags & 2)
            throw GdrError(GDR_ERR_BREAKDOWN, p.galerkin ? "FOM-DR-Sh: Ritz eigensolver did not converge"
                                                         : "GMRES-DR-Sh: harmonic Ritz eigensolver did not converge");
        const double r1 = (mixed ? rtn : o.snorm) / bnorm;
        double bmax = 1;
        for (int i = 1; i < ns; ++i) bmax = std::max(bmax, zabs(o.beta[i]));
        const double rmax = r1 * bmax;
        S.hist(0, cycles, mvps, o.snorm / bnorm, rmax);
        if (!std::isfinite(rmax))
            throw GdrError(GDR_ERR_BREAKDOWN, "GMRES-DR-Sh: non-finite residual norm");
        conv = rmax <= p.tol || brk >= 0;
        bool stop = conv;
        if (mixed && !conv) {
            // FP32 recursion has lost track of the true residual: leave the rest
            // to the FP64-refined cleanup
            const double gap = std::fabs(rtn - o.snorm) / rtn;
            if (rtn < 0.9 * best_true) {
                best_true = rtn;
                stall = 0;
            } else {
                ++stall;
            }
            if (gap > 0.5 || stall >= 3) stop = true;
        }
        if (brk >= 0) break;   // lucky breakdown: solved exactly, no deflation space
        S.theta(o.theta, k);
        S.prof.begin(GDR_K_RECOMBINE);
        vrecombine<T>(Vc, n, m + 1, P, m + 1, k + 1, Vn, n, n, st);
        S.prof.end(GDR_K_RECOMBINE, (double)n * (m + k + 2) * sizeof(C),
                   (double)n * (m + 1) * (k + 1) * 8);
        orth_column<T>(op, Vn, k, A.partial, A.nblk, tH, tcoef, tinv, tbrk);
        if (mixed) {
            // residual replacement: coordinates of the FP64 true residual in V_{k+1}
            gs_dot<T, double>(Vn, n, 0, k + 1, rtrue, 0, nullptr, 0, A.partial, A.nblk, n, 1, st);
            reduce_cols(A.partial, A.nblk, k + 2, tH, 0, nullptr, 0, 1, st);
            HIPCHK(hipMemcpyAsync(cx, tH, (k + 1) * sizeof(double2), hipMemcpyDeviceToDevice, st));
        }
        if (stop) break;
        std::swap(Vc, Vn);
        std::swap(Hc, Hx);
        std::swap(cc, cx);
        std::swap(cur, prv);
        j0 = k;
    }
    if (S.st) {
        S.st->cycles_dr += cycles;
        S.st->mvp_dr += mvps;
    }
    if (defl_out) {
        *defl_out = nullptr;
        if (brk < 0) {
            gdr_defl_s* d = new gdr_defl_s;
            d->op = op;
            d->k = k;
            d->prec = mixed ? GDR_PREC_MIXED : GDR_PREC_F64;
            try {
                HIPCHK(hipMalloc(&d->V, (size_t)(k + 1 + BASIS_PAD) * n * sizeof(C)));
                HIPCHK(hipMemsetAsync(d->V, 0, (size_t)(k + 1 + BASIS_PAD) * n * sizeof(C), st));
                HIPCHK(hipMemcpyAsync(d->V, Vn, (size_t)(k + 1) * n * sizeof(C),
                                      hipMemcpyDeviceToDevice, st));
                if (k > 0) {
                    HIPCHK(hipMalloc(&d->Hk, (size_t)(k + 1) * k * sizeof(double2)));
                    HIPCHK(hipMemcpy2DAsync(d->Hk, (k + 1) * sizeof(double2), Hx,
                                            (m + 1) * sizeof(double2), (k + 1) * sizeof(double2),
                                            k, hipMemcpyDeviceToDevice, st));
                    d->Hk_host.resize((size_t)(k + 1) * k);
                    HIPCHK(hipMemcpyAsync(d->Hk_host.data(), d->Hk,
                                          (size_t)(k + 1) * k * sizeof(double2),
                                          hipMemcpyDeviceToHost, st));
                }
                HIPCHK(hipStreamSynchronize(st));
            } catch (...) {
                delete d;
                throw;
            }
            *defl_out = d;
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    *conv_out = conv;
    return conv ? GDR_OK : GDR_NOT_CONVERGED;
}

int solve_dr_sh(gdr_op_s* op, int ns, const double2* sig, const double2* b_eo, double2* X_eo,
                const gdr_params& p, Stats& S, gdr_defl_s** defl_out, bool* converged) {
    if (p.precision == GDR_PREC_MIXED)
        return dr_run<float>(op, ns, sig, b_eo, X_eo, p, S, defl_out, converged);
    return dr_run<double>(op, ns, sig, b_eo, X_eo, p, S, defl_out, converged);
}

// ---------------------------------------------------------------------------
// GMRES-DR(m,k)-Sh on the first right-hand side of every lattice of a set
// (op->kind == 2), the lattices as the members of one batch: each member
// follows exactly the single-lattice algorithm of dr_run (its own Krylov
// space, harmonic Ritz restart, FP64 residual replacement and stopping
// rules); the operator of all members is one persistent work-list launch and
// every sweep is one launch over the members. Member b's right-hand side is
// b_eo + b*n and its ns solutions X + b*ns*n (n = the largest lattice's,
// zero beyond the member's own). The deflation pair of member b comes back in
// defl_out[b] for its own lattice (null after a lucky breakdown).
int solve_dr_many(gdr_op_s* op, int ns, const double2* sig_h, const double2* b_eo, double2* X,
                  const gdr_params& p, Stats& S, ManyOut& R) {
    using T = float;
    using C = typename CT<T>::t;
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    const int L = (int)op->parts.size();
    const int m = p.m_dr, k = p.k;
    DMem mem;
    const int64_t vms = (int64_t)(m + 1 + BASIS_PAD) * n;
    C* Va = alloc_basis<T>(mem, (m + 1 + BASIS_PAD) * L - BASIS_PAD, n, st);
    C* Vb = alloc_basis<T>(mem, (m + 1 + BASIS_PAD) * L - BASIS_PAD, n, st);
    Arnoldi<T> A;
    A.init(mem, op, m, L, Va, vms);
    A.use_graph = p.use_graph != 0;
    A.set_block(p.sstep, p.sstep_reorth);
    A.prof = &S.prof;
    const int64_t hms = A.hms;
    const int64_t pms = (int64_t)(m + 1) * (k + 1);
    const int64_t cms = (int64_t)(m + 1) * (ns + 1);
    double2* Hn = mem.get<double2>((size_t)hms * L);
    double2* c0 = mem.get<double2>((size_t)(m + 1) * L);
    double2* c1 = mem.get<double2>((size_t)(m + 1) * L);
    double2* coef = mem.get<double2>((size_t)cms * L);
    double2* P = mem.get<double2>((size_t)pms * L);
    CycleOut* outs = mem.get<CycleOut>((size_t)2 * L);
    double2* sig = mem.get<double2>(ns);
    double2* tG = mem.get<double2>((size_t)Arnoldi<T>::GMS * L);
    double2* tcoef = mem.get<double2>((size_t)GS_COEF_MS * L);
    double* tref = mem.get<double>(L);
    int* tbrk = mem.get<int>(L);
    double2* tH = mem.get<double2>((size_t)(k + 2) * L);
    double* dsc = mem.get<double>(L);
    int* act = mem.get<int>(L);
    double2* rtrue = mem.get<double2>((size_t)n * L);
    const int64_t bms = (int64_t)(sizeof(CycleOut) / sizeof(double2));
    HIPCHK(hipMemcpyAsync(sig, sig_h, ns * sizeof(double2), hipMemcpyHostToDevice, st));
    // rows beyond a member's own lattice are never written: zero once
    HIPCHK(hipMemsetAsync(rtrue, 0, (size_t)n * L * sizeof(double2), st));

    R.conv.assign(L, 0);
    R.cycles.assign(L, 0);
    R.mvps.assign(L, 0);
    R.defl.assign(L, nullptr);
    const std::vector<double> bnorm = norms_of(op, b_eo, L);
    for (int b = 0; b < L; ++b)
        if (!std::isfinite(bnorm[b])) throw GdrError(GDR_ERR_ARG, "right-hand side is not finite");
    HIPCHK(hipMemsetAsync(X, 0, (size_t)L * ns * n * sizeof(double2), st));
    std::vector<int> acth(L, 1);
    std::vector<CycleOut> init(L);
    std::vector<double2> ch((size_t)(m + 1) * L, z(0));
    std::vector<double> invb(L, 0);
    for (int b = 0; b < L; ++b) {
        init[b] = CycleOut{};
        init[b].snorm = bnorm[b];
        for (int i = 0; i < MAXNS; ++i) init[b].beta[i] = z(1);
        if (bnorm[b] > 0) {
            ch[(size_t)b * (m + 1)] = z(bnorm[b]);
            invb[b] = 1.0 / bnorm[b];
        } else {
            acth[b] = 0;   // b = 0: x = 0 is exact, no deflation space
            R.conv[b] = 1;
        }
    }
    HIPCHK(hipMemcpyAsync(outs, init.data(), L * sizeof(CycleOut), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c0, ch.data(), ch.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(dsc, invb.data(), L * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(Hn, 0, (size_t)hms * L * sizeof(double2), st));
    HIPCHK(hipMemsetAsync(A.H, 0, (size_t)hms * L * sizeof(double2), st));
    HIPCHK(hipMemcpyAsync(act, acth.data(), L * sizeof(int), hipMemcpyHostToDevice, st));
    convert_scale<T>(b_eo, n, dsc, 1, Va, vms, n, L, st, act);

    int cur = 1, prv = 0;
    C* Vc = Va;
    C* Vn = Vb;
    double2* Hc = A.H;
    double2* Hx = Hn;
    double2* cc = c0;
    double2* cx = c1;
    int j0 = 0;
    std::vector<double> best_true(L, std::numeric_limits<double>::infinity());
    std::vector<int> stall(L, 0), brkh(L, -1);
    std::vector<CycleOut> oh(L);
    const unsigned allx = ns >= 32 ? 0xffffffffu : ((1u << ns) - 1u);
    gdr_ctx_s* cx_ = op->ctx;
    for (int cyc = 0; cyc < p.max_cycles; ++cyc) {
        int nact = 0;
        for (int b = 0; b < L; ++b) nact += acth[b];
        if (nact == 0) break;
        A.V = Vc;
        A.H = Hc;
        A.cycle(j0, act, nact);
        HIPCHK(hipMemcpyAsync(outs + cur * L, init.data(), L * sizeof(CycleOut), hipMemcpyHostToDevice, st));
        CycleArgs a{};
        a.H = Hc;
        a.h_ms = hms;
        a.c = cc;
        a.c_ms = m + 1;
        a.sigma = sig;
        a.sig_ms = 0;
        a.beta = outs[prv * L].beta;
        a.beta_ms = bms;
        a.brk = A.brk;
        a.coef = coef;
        a.coef_ms = cms;
        a.out = outs + cur * L;
        a.restart = 0;
        a.k = k;
        a.P = P;
        a.p_ms = pms;
        a.Hnew = Hx;
        a.hnew_ms = hms;
        a.cnew = cx;
        a.cnew_ms = m + 1;
        a.m = m;
        a.ns = ns;
        a.act = act;
        a.galerkin = p.galerkin;
        S.prof.begin(GDR_K_SMALL);
        cycle_small(a, L, st);
        S.prof.end(GDR_K_SMALL, 0, 0);
        // the restart half on the auxiliary stream, overlapping the solution
        // update and the FP64 residuals (nothing below reads its outputs
        // before the join)
        HIPCHK(hipEventRecord(cx_->ev_fork, st));
        HIPCHK(hipStreamWaitEvent(cx_->aux, cx_->ev_fork, 0));
        {
            CycleArgs ar = a;
            ar.restart = 2;
            hipEvent_t pm = S.prof.mark(GDR_K_SMALL, cx_->aux);
            cycle_small(ar, L, cx_->aux);
            S.prof.span(GDR_K_SMALL, pm, cx_->aux, 0, 0);
        }
        HIPCHK(hipEventRecord(cx_->ev_join, cx_->aux));
        const double dn = (double)n * nact;
        S.prof.begin(GDR_K_COMBINE);
        vcombine<T>(Vc, n, vms, m, coef, m + 1, cms, ns, X, n, (int64_t)ns * n, allx, n, L, st, act);
        S.prof.end(GDR_K_COMBINE, dn * (m * sizeof(C) + 32.0 * ns), dn * m * ns * 8);
        {
            // FP64 true residuals of shift 1, each member on its own lattice
            DiagList dl{};
            for (int b = 0; b < L; ++b) {
                dl.d[b] = z(1.0 - sig_h[0].x, -sig_h[0].y);
                dl.alpha[b] = -1;
            }
            S.prof.begin(GDR_K_OTHER);
            op_apply<double>(op, X, (int64_t)ns * n, rtrue, n, b_eo, n, dl, L, st, act, 0);
            S.prof.end(GDR_K_OTHER, dslash_bytes<double>(op, nact, true), dslash_flops(op, nact));
            if (S.st) S.st->mvp_fp64 += nact;
        }
        HIPCHK(hipStreamWaitEvent(st, cx_->ev_join, 0));
        HIPCHK(hipMemcpyAsync(oh.data(), outs + cur * L, L * sizeof(CycleOut), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(brkh.data(), A.brk, L * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const std::vector<double> rtn = norms_of(op, rtrue, L);
        // per member: convergence, stall of the FP32 recursion, lucky breakdown
        std::vector<int> stop(L, 0), recomb(L, 0);
        double w1 = 0, wm = 0;
        int64_t mv = 0;
        for (int b = 0; b < L; ++b) {
            if (!acth[b]) continue;
            R.cycles[b] += 1;
            R.mvps[b] += m - j0;
            mv = std::max(mv, R.mvps[b]);
            if (oh[b].flags & 1)
                throw GdrError(GDR_ERR_BREAKDOWN, "GMRES-DR-Sh: singular shifted system ((Q^H s)_{m+1} = 0)");
            if (oh[b].flags & 2)
                throw GdrError(GDR_ERR_BREAKDOWN, "GMRES-DR-Sh: harmonic Ritz eigensolver did not converge");
            const double r1 = rtn[b] / bnorm[b];
            double bmax = 1;
            for (int i = 1; i < ns; ++i) bmax = std::max(bmax, zabs(oh[b].beta[i]));
            const double rmax = r1 * bmax;
            if (!std::isfinite(rmax)) throw GdrError(GDR_ERR_BREAKDOWN, "GMRES-DR-Sh: non-finite residual norm");
            w1 = std::max(w1, oh[b].snorm / bnorm[b]);
            wm = std::max(wm, rmax);
            const bool conv = rmax <= p.tol || brkh[b] >= 0;
            bool st_ = conv;
            if (!conv) {
                const double gap = std::fabs(rtn[b] - oh[b].snorm) / rtn[b];
                if (rtn[b] < 0.9 * best_true[b]) {
                    best_true[b] = rtn[b];
                    stall[b] = 0;
                } else {
                    ++stall[b];
                }
                if (gap > 0.5 || stall[b] >= 3) st_ = true;
            }
            R.conv[b] = conv ? 1 : 0;
            stop[b] = st_ || cyc + 1 >= p.max_cycles;
            recomb[b] = brkh[b] < 0;   // a lucky breakdown leaves no deflation space
        }
        S.hist(0, cyc + 1, mv, w1, wm);
        // restart of every member still active: V_{k+1} = V_{m+1} P, the last
        // column re-orthogonalised, the FP64 residual's coordinates in V_{k+1}
        S.prof.begin(GDR_K_RECOMBINE);
        for (int b = 0; b < L; ++b)
            if (acth[b] && recomb[b])
                vrecombine<T>(Vc + b * vms, n, m + 1, P + b * pms, m + 1, k + 1, Vn + b * vms, n, n, st);
        S.prof.end(GDR_K_RECOMBINE, dn * (m + k + 2) * sizeof(C), dn * (m + 1) * (k + 1) * 8);
        C* col = Vn + (int64_t)k * n;
        for (int pass = 0; pass < 2; ++pass) {
            fill_int(tbrk, -1, L, st);
            gs_dot<T, T>(Vn, n, vms, k + 1, col, vms, (const C*)nullptr, 0, A.partial, A.nblk, n, L, st,
                         act);
            reduce_cols(A.partial, A.nblk, k + 2, tG, Arnoldi<T>::GMS, nullptr, 0, L, st, act);
            dcgs_coef(tG, Arnoldi<T>::GMS, k, 1, 1, nullptr, 0, 0, tcoef, GS_COEF_MS, tref, tbrk, 0.0, L,
                      st, act);
            gs_update<T>(Vn, n, vms, k, col, vms, (const C*)nullptr, 0, col, vms, (C*)nullptr, 0, tcoef,
                         GS_COEF_MS, n, L, st, act);
        }
        gs_dot<T, double>(Vn, n, vms, k + 1, rtrue, n, nullptr, 0, A.partial, A.nblk, n, L, st, act);
        reduce_cols(A.partial, A.nblk, k + 2, tH, k + 2, nullptr, 0, L, st, act);
        HIPCHK(hipMemcpy2DAsync(cx, (m + 1) * sizeof(double2), tH, (k + 2) * sizeof(double2),
                                (k + 1) * sizeof(double2), L, hipMemcpyDeviceToDevice, st));
        // members that stop: their deflation pair, then they leave the batch
        bool changed = false;
        for (int b = 0; b < L; ++b) {
            if (!acth[b] || !stop[b]) continue;
            changed = true;
            acth[b] = 0;
            if (!recomb[b]) continue;
            gdr_op_s* q = op->parts[b];
            const int64_t nq = q->n;
            gdr_defl_s* d = new gdr_defl_s;
            d->op = q;
            d->k = k;
            d->prec = GDR_PREC_MIXED;
            R.defl[b] = d;
            HIPCHK(hipMalloc(&d->V, (size_t)(k + 1 + BASIS_PAD) * nq * sizeof(C)));
            HIPCHK(hipMemsetAsync(d->V, 0, (size_t)(k + 1 + BASIS_PAD) * nq * sizeof(C), st));
            HIPCHK(hipMemcpy2DAsync(d->V, nq * sizeof(C), Vn + b * vms, n * sizeof(C), nq * sizeof(C),
                                    k + 1, hipMemcpyDeviceToDevice, st));
            if (k > 0) {
                HIPCHK(hipMalloc(&d->Hk, (size_t)(k + 1) * k * sizeof(double2)));
                HIPCHK(hipMemcpy2DAsync(d->Hk, (k + 1) * sizeof(double2), Hx + b * hms,
                                        (m + 1) * sizeof(double2), (k + 1) * sizeof(double2), k,
                                        hipMemcpyDeviceToDevice, st));
                d->Hk_host.resize((size_t)(k + 1) * k);
                HIPCHK(hipMemcpyAsync(d->Hk_host.data(), d->Hk, (size_t)(k + 1) * k * sizeof(double2),
                                      hipMemcpyDeviceToHost, st));
            }
        }
        if (changed) {
            HIPCHK(hipMemcpyAsync(act, acth.data(), L * sizeof(int), hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        std::swap(Vc, Vn);
        std::swap(Hc, Hx);
        std::swap(cc, cx);
        std::swap(cur, prv);
        j0 = k;
    }
    HIPCHK(hipStreamSynchronize(st));
    if (S.st) {
        for (int b = 0; b < L; ++b) {
            S.st->cycles_dr += R.cycles[b];
            S.st->mvp_dr += R.mvps[b];
        }
    }
    for (int b = 0; b < L; ++b)
        if (!R.conv[b]) return GDR_NOT_CONVERGED;
    return GDR_OK;
}

// ---------------------------------------------------------------------------
// GMRES(m)-Proj(k)-Sh over a batch of members (Sec. 4, GMRES-Proj-Sh steps
// 2-6). Member b solves (A - sig[b][i]) x_i = B[b] for i < ns; its state
// block W[b] holds x_0 .. x_{ns-1} and the base residual r (FP64).
struct ProjResult {
    std::vector<int64_t> mvps;
    std::vector<int> cycles;
    std::vector<int> conv;
    std::vector<double2> beta, gam;   // at the end, per member ns
};

template <typename T>
static void proj_run(gdr_op_s* op, gdr_defl_s* defl, int nmem, int ns,
                     const std::vector<double2>& sig_h, const double2* Bm, double2* W,
                     const std::vector<double>& tol, const std::vector<double>& bnorm, int m,
                     int max_cycles, Stats& S, const std::vector<int>& phase, ProjResult& R,
                     bool start = false, int kp = 0, bool graph = false, int sblk = 0,
                     double reorth = 20, bool replace = true) {
    // kp > 0: project over the leading kp deflation vectors only (the
    // accurate-eigenvector variant, Table 4.1); otherwise over all k.
    // replace (mixed precision): the base residual is replaced by the FP64
    // true residual after every cycle; otherwise the FP32 recursion's residual
    // is kept (inner solves of a refinement, whose caller checks true residuals)
    // graph: replay the Arnoldi cycle from a captured HIP graph
    // start: W already holds an initial guess x_i and the common residual r
    // (related right-hand sides, Sec. 5); otherwise x_i = 0, r = b
    using C = typename CT<T>::t;
    constexpr bool mixed = std::is_same<T, float>::value;
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    const int k = defl ? defl->k : 0;
    const C* Vd = defl ? (const C*)defl->V : nullptr;
    DMem mem;
    const int64_t vms = (int64_t)(m + 1 + BASIS_PAD) * n;
    const int64_t wms = (int64_t)(ns + 1) * n;
    C* Vb = alloc_basis<T>(mem, (m + 1 + BASIS_PAD) * nmem - BASIS_PAD, n, st);
    Arnoldi<T> A;
    A.init(mem, op, m, nmem, Vb, vms);
    A.use_graph = graph;
    A.set_block(sblk, reorth);
    A.prof = &S.prof;
    double2* sig = mem.get<double2>((size_t)nmem * ns);
    double2* Cb = mem.get<double2>((size_t)80 * nmem);
    double2* cvec = mem.get<double2>((size_t)(m + 1) * nmem);
    const int64_t cpms = (int64_t)(k + 1) * (ns + 1);
    const int64_t ccms = (int64_t)(m + 1) * (ns + 1);
    double2* coefP = mem.get<double2>((size_t)cpms * nmem);
    double2* coefC = mem.get<double2>((size_t)ccms * nmem);
    double2* gam = mem.get<double2>((size_t)ns * nmem);
    double2* rn2 = mem.get<double2>((size_t)nmem);
    CycleOut* outs = mem.get<CycleOut>((size_t)2 * nmem);
    int* act = mem.get<int>(nmem);
    int* pflags = mem.get<int>(nmem);
    const int64_t bms = (int64_t)(sizeof(CycleOut) / sizeof(double2));
    static_assert(sizeof(CycleOut) % sizeof(double2) == 0, "CycleOut layout");

    HIPCHK(hipMemcpyAsync(sig, sig_h.data(), (size_t)nmem * ns * sizeof(double2),
                          hipMemcpyHostToDevice, st));
    if (!start) {
        HIPCHK(hipMemsetAsync(W, 0, (size_t)wms * nmem * sizeof(double2), st));
        copy_vec(Bm, n, W + (int64_t)ns * n, wms, n, nmem, st);   // r = b
    }
    std::vector<CycleOut> init(2 * nmem);
    for (auto& o : init) {
        o = CycleOut{};
        for (int i = 0; i < MAXNS; ++i) o.beta[i] = z(1);
    }
    HIPCHK(hipMemcpyAsync(outs, init.data(), 2 * nmem * sizeof(CycleOut), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(gam, 0, (size_t)ns * nmem * sizeof(double2), st));
    HIPCHK(hipMemsetAsync(pflags, 0, nmem * sizeof(int), st));
    HIPCHK(hipMemsetAsync(A.H, 0, (size_t)A.hms * nmem * sizeof(double2), st));
    std::vector<int> acth(nmem, 1);
    HIPCHK(hipMemcpyAsync(act, acth.data(), nmem * sizeof(int), hipMemcpyHostToDevice, st));

    R.mvps.assign(nmem, 0);
    R.cycles.assign(nmem, 0);
    R.conv.assign(nmem, 0);
    R.beta.assign((size_t)nmem * ns, z(1));
    R.gam.assign((size_t)nmem * ns, z(0));
    const unsigned keep_all = (1u << (ns + 1)) - 1u;
    const unsigned keep_x = (1u << ns) - 1u;
    int cur = 1, prv = 0;
    std::vector<CycleOut> oh(nmem);
    std::vector<double2> rnh(nmem);
    const double cs = sizeof(C);
    for (int cyc = 0; cyc < max_cycles; ++cyc) {
        int nact0 = 0;
        for (int b = 0; b < nmem; ++b) nact0 += acth[b];
        const double dn = (double)n * nact0;
        // ---- minres projection over V_k with v_{k+1} tracking
        if (k > 0) {
            // every member projects on the one deflation basis V_{k+1}
            if (k + 1 <= SHARED_NC_MAX)
                shared_dot<T, double>(Vd, n, k + 1, W + (int64_t)ns * n, wms, A.partial, A.nblk,
                                      n, nmem, st, act);
            else
                gs_dot<T, double>(Vd, n, 0, k + 1, W + (int64_t)ns * n, wms, nullptr, 0,
                                  A.partial, A.nblk, n, nmem, st, act);
            reduce_cols(A.partial, A.nblk, k + 2, Cb, 80, nullptr, 0, nmem, st, act);
            ProjArgs pa{};
            pa.Hk = defl->Hk;
            pa.k = k;
            pa.kp = (kp > 0 && kp < k) ? kp : k;
            pa.C = Cb;
            pa.c_ms = 80;
            pa.sigma = sig;
            pa.sig_ms = ns;
            pa.beta = outs[prv * nmem].beta;
            pa.beta_ms = bms;
            pa.gam = gam;
            pa.gam_ms = ns;
            pa.coef = coefP;
            pa.coef_ms = cpms;
            pa.flags = pflags;
            pa.ns = ns;
            pa.act = act;
            S.prof.begin(GDR_K_SMALL);
            proj_small(pa, nmem, st);
            S.prof.end(GDR_K_SMALL, 0, 0);
            S.prof.begin(GDR_K_COMBINE);
            vcombine<T>(Vd, n, 0, k + 1, coefP, k + 1, cpms, ns + 1, W, n, wms, keep_all, n, nmem,
                        st, act);
            S.prof.end(GDR_K_COMBINE, dn * ((k + 1) * cs + 32.0 * (ns + 1)),
                       dn * (k + 1) * (ns + 1) * 8);
        }
        // ---- one GMRES(m)-Sh cycle from r
        gs_dot<double, double>(nullptr, 0, 0, 0, W + (int64_t)ns * n, wms, nullptr, 0, A.partial,
                               A.nblk, n, nmem, st, act);
        reduce_cols(A.partial, A.nblk, 1, rn2, 1, nullptr, 0, nmem, st, act);
        start_cycle(rn2, 1, cvec, m + 1, m, A.inv, nmem, st, act);
        convert_scale<T>(W + (int64_t)ns * n, wms, A.inv, 1, Vb, vms, n, nmem, st, act);
        A.cycle(0, act, nact0);
        HIPCHK(hipMemcpyAsync(outs + cur * nmem, init.data(), nmem * sizeof(CycleOut),
                              hipMemcpyHostToDevice, st));
        CycleArgs a{};
        a.H = A.H;
        a.h_ms = A.hms;
        a.c = cvec;
        a.c_ms = m + 1;
        a.sigma = sig;
        a.sig_ms = ns;
        a.beta = outs[prv * nmem].beta;
        a.beta_ms = bms;
        a.brk = A.brk;
        a.coef = coefC;
        a.coef_ms = ccms;
        a.out = outs + cur * nmem;
        a.restart = 0;
        a.k = 0;
        a.m = m;
        a.ns = ns;
        a.act = act;
        S.prof.begin(GDR_K_SMALL);
        cycle_small(a, nmem, st);
        S.prof.end(GDR_K_SMALL, 0, 0);
        // x_i += V_m d_i ; r = V_{m+1} s
        S.prof.begin(GDR_K_COMBINE);
        vcombine<T>(Vb, n, vms, m + 1, coefC, m + 1, ccms, ns + 1, W, n, wms, keep_x, n, nmem, st,
                    act);
        S.prof.end(GDR_K_COMBINE, dn * ((m + 1) * cs + 32.0 * ns + 16),
                   dn * (m + 1) * (ns + 1) * 8);
        if (mixed && replace) {
            // base residual replaced by the FP64 true residual of shift 1
            for (int b0 = 0; b0 < nmem; b0 += DSLASH_MAXV) {
                const int nb = std::min(DSLASH_MAXV, nmem - b0);
                DiagList dl{};
                for (int v = 0; v < nb; ++v) {
                    const double2 s1 = sig_h[(size_t)(b0 + v) * ns];
                    dl.d[v] = z(1.0 - s1.x, -s1.y);
                    dl.alpha[v] = -1;
                }
                const int na = std::min(nb, nact0 - std::min(nact0, b0));
                S.prof.begin(GDR_K_OTHER);   // FP64 true residuals
                op_apply<double>(op, W + b0 * wms, wms, W + b0 * wms + (int64_t)ns * n, wms,
                               Bm + b0 * n, n, dl, nb,
                               st, act + b0);
                S.prof.end(GDR_K_OTHER, dslash_bytes<double>(op, na, true), dslash_flops(op, na));
                if (S.st) S.st->mvp_fp64 += na;
            }
            gs_dot<double, double>(nullptr, 0, 0, 0, W + (int64_t)ns * n, wms, nullptr, 0,
                                   A.partial, A.nblk, n, nmem, st, act);
            reduce_cols(A.partial, A.nblk, 1, rn2, 1, nullptr, 0, nmem, st, act);
            HIPCHK(hipMemcpyAsync(rnh.data(), rn2, nmem * sizeof(double2), hipMemcpyDeviceToHost, st));
        }
        HIPCHK(hipMemcpyAsync(oh.data(), outs + cur * nmem, nmem * sizeof(CycleOut),
                              hipMemcpyDeviceToHost, st));
        int pf_any = 0;
        std::vector<int> pfl(nmem);
        HIPCHK(hipMemcpyAsync(pfl.data(), pflags, nmem * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        int nact = 0;
        double worst = 0, worst_r1 = 0;
        int64_t step_mvps = 0;
        for (int b = 0; b < nmem; ++b) {
            if (!acth[b]) continue;
            pf_any |= pfl[b];
            if (oh[b].flags) pf_any |= 4;
            R.mvps[b] += m;
            step_mvps += m;
            R.cycles[b] += 1;
            const double rn = mixed && replace ? std::sqrt(rnh[b].x) : oh[b].snorm;
            double bmax = 1;
            for (int i = 1; i < ns; ++i) bmax = std::max(bmax, zabs(oh[b].beta[i]));
            const double r1 = rn / bnorm[b];
            const double rmax = r1 * bmax;
            if (!std::isfinite(rmax))
                throw GdrError(GDR_ERR_BREAKDOWN, "GMRES-Proj-Sh: non-finite residual norm");
            worst = std::max(worst, rmax);
            worst_r1 = std::max(worst_r1, r1);
            for (int i = 0; i < ns; ++i) R.beta[(size_t)b * ns + i] = oh[b].beta[i];
            if (rmax <= tol[b]) {
                acth[b] = 0;
                R.conv[b] = 1;
            } else {
                ++nact;
            }
        }
        if (pf_any & 1) throw GdrError(GDR_ERR_BREAKDOWN, "GMRES-Proj-Sh: singular H_k - sigma_i I");
        if (pf_any & 4) throw GdrError(GDR_ERR_BREAKDOWN, "GMRES-Proj-Sh: singular shifted system in a GMRES-Sh cycle");
        // history: one record per distinct phase of the batch (max over its members)
        {
            std::vector<int> seen;
            for (int b = 0; b < nmem; ++b) {
                if (std::find(seen.begin(), seen.end(), phase[b]) != seen.end()) continue;
                seen.push_back(phase[b]);
                double w1 = 0, wm = 0;
                int64_t mv = 0;
                bool any = false;
                for (int c = 0; c < nmem; ++c)
                    if (phase[c] == phase[b] && R.cycles[c] == cyc + 1) {
                        any = true;
                        const double rn = mixed && replace ? std::sqrt(rnh[c].x) : oh[c].snorm;
                        double bmax = 1;
                        for (int i = 1; i < ns; ++i) bmax = std::max(bmax, zabs(oh[c].beta[i]));
                        w1 = std::max(w1, rn / bnorm[c]);
                        wm = std::max(wm, bmax * rn / bnorm[c]);
                        mv = std::max(mv, R.mvps[c]);
                    }
                if (any) S.hist(phase[b], cyc + 1, mv, w1, wm);
            }
        }
        (void)worst;
        (void)worst_r1;
        (void)step_mvps;
        HIPCHK(hipMemcpyAsync(act, acth.data(), nmem * sizeof(int), hipMemcpyHostToDevice, st));
        std::swap(cur, prv);
        if (nact == 0) break;
    }
    std::vector<double2> gh((size_t)nmem * ns);
    HIPCHK(hipMemcpyAsync(gh.data(), gam, gh.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    R.gam = gh;
}

// T -> FP64 copy of the defl's v_{k+1}
template <typename T>
static void vk1_to_f64(gdr_defl_s* d, double2* out) {
    using C = typename CT<T>::t;
    gdr_op_s* op = d->op;
    DMem mem;
    double2* one = mem.get<double2>(1);
    const double2 o = z(1);
    HIPCHK(hipMemcpyAsync(one, &o, sizeof(o), hipMemcpyHostToDevice, op->ctx->st));
    vcombine<T>((const C*)d->V + (int64_t)d->k * op->n, op->n, 0, 1, one, 1, 0, 1, out, op->n, 0,
                0u, op->n, 1, op->ctx->st);
    HIPCHK(hipStreamSynchronize(op->ctx->st));
}

// gamma_hat_i = v_{k+1}^H (rhs - (A - sigma_i) x_i) for i = 1..ns-1 of one
// member; returns host values (index i-1) and leaves nothing else changed.
template <typename T>
static std::vector<double2> vk1_dot_residuals(gdr_defl_s* d, int ns, const double2* sig_h,
                                              const double2* xs, const double2* rhs,
                                              double2* Rt, double2* part, int nblk, double2* g) {
    using C = typename CT<T>::t;
    gdr_op_s* op = d->op;
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    DiagList dl{};
    for (int i = 1; i < ns; ++i) {
        dl.d[i - 1] = z(1.0 - sig_h[i].x, -sig_h[i].y);
        dl.alpha[i - 1] = -1;
    }
    op_apply<double>(op, xs + n, n, Rt, n, rhs, 0, dl, ns - 1,
                   st);
    gs_dot<T, double>((const C*)d->V + (int64_t)d->k * n, n, 0, 1, Rt, n, nullptr, 0, part, nblk,
                      n, ns - 1, st);
    reduce_cols(part, nblk, 2, g, 2, nullptr, 0, ns - 1, st);
    std::vector<double2> gh(2 * (ns - 1));
    HIPCHK(hipMemcpyAsync(gh.data(), g, gh.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<double2> out(ns - 1);
    for (int i = 0; i < ns - 1; ++i) out[i] = gh[2 * i];
    return out;
}

// Related right-hand sides (Sec. 5, eq. (5.2)): project member b's right-hand
// side over the earlier ones, Bp = [b^1 .. b^np] (the most recent MAXM):
// (Bp^H Bp) d = Bp^H b (shift independent), x_i = X_i^{prev} d for every
// shift, and the common residual r = b - Bp d, written into W (member block
// [x_1 .. x_ns, r]). The extra right-hand side (id < 0) starts from zero.
static void related_start(gdr_op_s* op, int ns, const double2* Ball, const double2* Xall,
                          int nsolved, const std::vector<int>& ids, const double2* Bm, double2* W,
                          hipStream_t st) {
    const int64_t n = op->n;
    const int nmem = (int)ids.size();
    const int64_t wms = (int64_t)(ns + 1) * n;
    const int np = std::min(nsolved, MAXM);
    const double2* Bp = Ball + (int64_t)(nsolved - np) * n;
    const double2* Xp = Xall + (int64_t)(nsolved - np) * ns * n;
    DMem mem;
    const int nblk = cgs_nblk(n);
    double2* part = mem.get<double2>((size_t)(np + 1) * nblk * std::max(np, nmem));
    double2* G = mem.get<double2>((size_t)(np + 1) * np);
    double2* g = mem.get<double2>((size_t)(np + 1) * nmem);
    double2* dv = mem.get<double2>((size_t)np * nmem);
    double2* dn = mem.get<double2>((size_t)np * nmem);
    // G column l = Bp^H b^l; g_b = Bp^H b_b (each with a norm slot, ignored);
    // one shared basis Bp for all columns
    if (np <= SHARED_NC_MAX) {
        shared_dot<double, double>(Bp, n, np, Bp, n, part, nblk, n, np, st);
        reduce_cols(part, nblk, np + 1, G, np + 1, nullptr, 0, np, st);
        shared_dot<double, double>(Bp, n, np, Bm, n, part, nblk, n, nmem, st);
    } else {
        gs_dot<double, double>(Bp, n, 0, np, Bp, n, nullptr, 0, part, nblk, n, np, st);
        reduce_cols(part, nblk, np + 1, G, np + 1, nullptr, 0, np, st);
        gs_dot<double, double>(Bp, n, 0, np, Bm, n, nullptr, 0, part, nblk, n, nmem, st);
    }
    reduce_cols(part, nblk, np + 1, g, np + 1, nullptr, 0, nmem, st);
    // compact G to ld np
    double2* Gc = mem.get<double2>((size_t)np * np);
    for (int l = 0; l < np; ++l)
        HIPCHK(hipMemcpyAsync(Gc + (int64_t)l * np, G + (int64_t)l * (np + 1), np * sizeof(double2),
                              hipMemcpyDeviceToDevice, st));
    gram_solve(Gc, np, g, np + 1, dv, dn, np, nmem, st);
    HIPCHK(hipMemsetAsync(W, 0, (size_t)wms * nmem * sizeof(double2), st));
    copy_vec(Bm, n, W + (int64_t)ns * n, wms, n, nmem, st);
    std::vector<int> acth(nmem);
    for (int b = 0; b < nmem; ++b) acth[b] = ids[b] >= 0;
    int* act = mem.get<int>(nmem);
    HIPCHK(hipMemcpyAsync(act, acth.data(), nmem * sizeof(int), hipMemcpyHostToDevice, st));
    // x_i = sum_l d_l x_i^l  (previous solutions of shift i are ns*n apart)
    for (int i = 0; i < ns; ++i)
        vcombine<double>(Xp + (int64_t)i * n, (int64_t)ns * n, 0, np, dv, np, np, 1, W + (int64_t)i * n,
                         n, wms, 0u, n, nmem, st, act);
    // r = b - Bp d
    vcombine<double>(Bp, n, 0, np, dn, np, np, 1, W + (int64_t)ns * n, n, wms, 1u, n, nmem, st, act);
    HIPCHK(hipStreamSynchronize(st));
}

// Later right-hand sides B_eo[0..nrhs) (and the extra right-hand side when
// needed) by GMRES-Proj-Sh with the correction. The nprev right-hand sides
// stored just before B_eo (and their solutions just before X_eo) are already
// solved; with p.related_rhs every batch first projects over all right-hand
// sides solved before it (Sec. 5, eq. (5.2)).
template <typename T>
static int proj_batch(gdr_op_s* op, gdr_defl_s* d, int ns, const double2* sig_h, int nrhs,
                      const double2* B_eo, double2* X_eo, int nprev, const gdr_params& p,
                      Stats& S) {
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    const int m = p.m_proj;
    const double tol_extra = p.tol_extra > 0 ? p.tol_extra : std::sqrt(p.tol);
    const int kp = std::min(p.proj_k, d->k);   // > 0: accurate-eigenvector variant
    bool need_extra = ns > 1 && d->k > 0 && kp == 0;
    if (need_extra && d->S && (int)d->extra_sig.size() == ns) {
        need_extra = false;
        for (int i = 0; i < ns; ++i)
            if (d->extra_sig[i].x != sig_h[i].x || d->extra_sig[i].y != sig_h[i].y) need_extra = true;
    }
    const int chunk = p.batch ? 16 : 1;
    DMem mem;
    const int nblk = cgs_nblk(n);
    double2* Rt = mem.get<double2>((size_t)std::max(ns - 1, 1) * n);
    double2* part = mem.get<double2>((size_t)2 * nblk * std::max(ns, 1));
    double2* g = mem.get<double2>((size_t)2 * std::max(ns, 1));
    double2* fac = mem.get<double2>(std::max(ns, 1));
    std::vector<double2> sigl(sig_h, sig_h + ns);
    bool all_conv = true;
    // members: -1 = extra right-hand side, 0..nrhs-1 = B columns
    std::vector<int> todo;
    if (need_extra) todo.push_back(-1);
    for (int j = 0; j < nrhs; ++j) todo.push_back(j);
    size_t pos = 0;
    while (pos < todo.size()) {
        const int nmem = (int)std::min<size_t>(chunk, todo.size() - pos);
        std::vector<int> ids(todo.begin() + pos, todo.begin() + pos + nmem);
        pos += nmem;
        DMem cm;
        double2* Bm = cm.get<double2>((size_t)nmem * n);
        double2* W = cm.get<double2>((size_t)nmem * (ns + 1) * n);
        std::vector<double> tol(nmem), bnorm(nmem);
        std::vector<int> phase(nmem);
        std::vector<double2> sgm((size_t)nmem * ns);
        for (int b = 0; b < nmem; ++b) {
            if (ids[b] < 0) {
                if (d->prec == GDR_PREC_MIXED) vk1_to_f64<float>(d, Bm + b * n);
                else vk1_to_f64<double>(d, Bm + b * n);
                tol[b] = tol_extra;
                phase[b] = 1;
            } else {
                HIPCHK(hipMemcpyAsync(Bm + b * n, B_eo + (int64_t)ids[b] * n, n * sizeof(double2),
                                      hipMemcpyDeviceToDevice, st));
                tol[b] = p.tol;
                phase[b] = 2 + ids[b];
            }
            bnorm[b] = vec_norm(op, Bm + b * n);
            if (!std::isfinite(bnorm[b]))
                throw GdrError(GDR_ERR_ARG, "right-hand side is not finite");
            if (!(bnorm[b] > 0)) bnorm[b] = 1;
            for (int i = 0; i < ns; ++i) sgm[(size_t)b * ns + i] = sig_h[i];
        }
        ProjResult R;
        using clock = std::chrono::steady_clock;
        auto t0 = clock::now();
        // right-hand sides solved before this batch: the nprev given ones and
        // the earlier batches' (their solutions are final: corrected below)
        int first_b = -1;
        for (int b = 0; b < nmem; ++b)
            if (ids[b] >= 0) {
                first_b = ids[b];
                break;
            }
        const int nsolved = first_b >= 0 ? nprev + first_b : 0;
        const bool related = p.related_rhs && nsolved > 0;
        if (related) related_start(op, ns, B_eo - (int64_t)nprev * n, X_eo - (int64_t)nprev * ns * n,
                                   nsolved, ids, Bm, W, st);
        if (d->prec == GDR_PREC_MIXED)
            proj_run<float>(op, d, nmem, ns, sgm, Bm, W, tol, bnorm, m, p.max_cycles, S, phase, R,
                            related, kp, p.use_graph != 0, p.sstep, p.sstep_reorth);
        else
            proj_run<double>(op, d, nmem, ns, sgm, Bm, W, tol, bnorm, m, p.max_cycles, S, phase, R,
                             related, kp, p.use_graph != 0);
        HIPCHK(hipStreamSynchronize(st));
        auto t1 = clock::now();
        if (S.st) S.st->t_phase[2] += std::chrono::duration<double>(t1 - t0).count();
        const int64_t wms = (int64_t)(ns + 1) * n;
        for (int b = 0; b < nmem; ++b) {
            if (ids[b] < 0) {
                if (S.st) {
                    S.st->mvp_extra += R.mvps[b];
                    S.st->cycles_extra += R.cycles[b];
                }
                d->mvp_extra = R.mvps[b];
                d->cycles_extra = R.cycles[b];
            } else if (S.st) {
                S.st->mvp_proj += R.mvps[b];
                S.st->cycles_proj += R.cycles[b];
            }
            if (!R.conv[b]) all_conv = false;
        }
        auto t2 = clock::now();
        // ---- extra right-hand side correction: s_i = s~_i / (1 - gamma_i)
        for (int b = 0; b < nmem; ++b) {
            if (ids[b] >= 0) continue;
            double2* xs = W + b * wms;
            auto gh = d->prec == GDR_PREC_MIXED
                          ? vk1_dot_residuals<float>(d, ns, sig_h, xs, Bm + b * n, Rt, part, nblk, g)
                          : vk1_dot_residuals<double>(d, ns, sig_h, xs, Bm + b * n, Rt, part, nblk, g);
            if (S.st) S.st->mvp_fp64 += ns - 1;
            std::vector<double2> f(ns, z(1));
            for (int i = 1; i < ns; ++i) {
                const double2 om = z(1.0 - gh[i - 1].x, -gh[i - 1].y);
                const double den = om.x * om.x + om.y * om.y;
                if (!(std::sqrt(den) > 1e-12))
                    throw GdrError(GDR_ERR_BREAKDOWN, "extra right-hand side: 1 - gamma_i = 0");
                f[i] = z(om.x / den, -om.y / den);
            }
            if (!d->S) HIPCHK(hipMalloc(&d->S, (size_t)ns * n * sizeof(double2)));
            else if ((int)d->extra_sig.size() < ns) {
                (void)hipFree(d->S);
                d->S = nullptr;
                HIPCHK(hipMalloc(&d->S, (size_t)ns * n * sizeof(double2)));
            }
            HIPCHK(hipMemcpyAsync(d->S, xs, (size_t)ns * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(fac, f.data(), ns * sizeof(double2), hipMemcpyHostToDevice, st));
            scal_dev(d->S + n, n, fac + 1, n, ns - 1, st);
            d->extra_sig = sigl;
            HIPCHK(hipStreamSynchronize(st));
        }
        // ---- correction of every right-hand side: x_i += (v_{k+1}^H r_i) s_i
        for (int b = 0; b < nmem; ++b) {
            if (ids[b] < 0) continue;
            double2* xs = W + b * wms;
            if (ns > 1 && d->k > 0 && kp == 0) {
                auto gh = d->prec == GDR_PREC_MIXED
                              ? vk1_dot_residuals<float>(d, ns, sig_h, xs, Bm + b * n, Rt, part, nblk, g)
                              : vk1_dot_residuals<double>(d, ns, sig_h, xs, Bm + b * n, Rt, part, nblk, g);
                if (S.st) S.st->mvp_fp64 += ns - 1;
                HIPCHK(hipMemcpyAsync(fac, gh.data(), (ns - 1) * sizeof(double2), hipMemcpyHostToDevice, st));
                axpy_dev(xs + n, n, d->S + n, n, fac, 1, n, ns - 1, st);
            }
            HIPCHK(hipMemcpyAsync(X_eo + (int64_t)ids[b] * ns * n, xs, (size_t)ns * n * sizeof(double2),
                                  hipMemcpyDeviceToDevice, st));
        }
        HIPCHK(hipStreamSynchronize(st));
        auto t3 = clock::now();
        if (S.st) S.st->t_phase[3] += std::chrono::duration<double>(t3 - t2).count();
    }
    return all_conv ? GDR_OK : GDR_NOT_CONVERGED;
}

int solve_proj_batch(gdr_op_s* op, gdr_defl_s* defl, int ns, const double2* sig, int nrhs,
                     const double2* B_eo, double2* X_eo, int nprev, const gdr_params& p, Stats& S) {
    if (defl->prec == GDR_PREC_MIXED)
        return proj_batch<float>(op, defl, ns, sig, nrhs, B_eo, X_eo, nprev, p, S);
    return proj_batch<double>(op, defl, ns, sig, nrhs, B_eo, X_eo, nprev, p, S);
}

// ---------------------------------------------------------------------------
static void residual_vectors(gdr_op_s* op, int ns, const double2* sig, const double2* b,
                             const double2* xs, double2* R) {
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    for (int i0 = 0; i0 < ns; i0 += DSLASH_MAXV) {
        const int nb = std::min(DSLASH_MAXV, ns - i0);
        DiagList dl{};
        for (int v = 0; v < nb; ++v) {
            dl.d[v] = z(1.0 - sig[i0 + v].x, -sig[i0 + v].y);
            dl.alpha[v] = -1;
        }
        op_apply<double>(op, xs + (int64_t)i0 * n, n, R + (int64_t)i0 * n, n, b, 0, dl, nb, st);
    }
}

std::vector<double> norms_of(gdr_op_s* op, const double2* R, int nv) {
    hipStream_t st = op->ctx->st;
    DMem mem;
    const int nblk = cgs_nblk(op->n);
    double2* part = mem.get<double2>((size_t)nblk * nv);
    double2* out = mem.get<double2>(nv);
    gs_dot<double, double>(nullptr, 0, 0, 0, R, op->n, nullptr, 0, part, nblk, op->n, nv, st);
    reduce_cols(part, nblk, 1, out, 1, nullptr, 0, nv, st);
    std::vector<double2> h(nv);
    HIPCHK(hipMemcpyAsync(h.data(), out, nv * sizeof(double2), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<double> r(nv);
    for (int i = 0; i < nv; ++i) r[i] = std::sqrt(h[i].x);
    return r;
}

void true_residuals(gdr_op_s* op, int ns, const double2* sig, int nrhs, const double2* B_eo,
                    const double2* X_eo, std::vector<double>& resid) {
    DMem mem;
    const int64_t n = op->n;
    double2* R = mem.get<double2>((size_t)ns * n);
    resid.assign((size_t)nrhs * ns, 0);
    for (int j = 0; j < nrhs; ++j) {
        const double bn = vec_norm(op, B_eo + (int64_t)j * n);
        residual_vectors(op, ns, sig, B_eo + (int64_t)j * n, X_eo + (int64_t)j * ns * n, R);
        auto rn = norms_of(op, R, ns);
        for (int i = 0; i < ns; ++i) resid[(size_t)j * ns + i] = bn > 0 ? rn[i] / bn : rn[i];
    }
}

int cleanup(gdr_op_s* op, gdr_defl_s* defl, int ns, const double2* sig, int nrhs,
            const double2* B_eo, double2* X_eo, const gdr_params& p, Stats& S) {
    // the refinement solves apply the operator with FP32 links even where the
    // Krylov phases used FP16-stored ones
    RefineLinks fp32_links(op);
    hipStream_t st = op->ctx->st;
    const int64_t n = op->n;
    DMem mem;
    double2* R = mem.get<double2>((size_t)ns * n);
    std::vector<double> bn(nrhs);
    for (int j = 0; j < nrhs; ++j) bn[j] = vec_norm(op, B_eo + (int64_t)j * n);
    bool done = false;
    // the residuals left by the FP32 phases are already small and the
    // deflation space is reused: short cycles reach the needed reduction
    // (8 measured fastest on the 24^3x48 twelve-RHS workload: 16 and 24 cost
    // 1.7x and 6x more cleanup time for the same final residuals)
    const int mc = p.m_clean > 0 ? p.m_clean : std::min(p.m_proj, 8);
    // The inner solves keep the FP32 recursion's residual (no FP64
    // replacement per cycle): they only reduce their residual by a factor of
    // at least 1e-5, well within what the recursion tracks, and every round
    // starts from FP64 true residuals (24^3x48: the same products, -8 % of
    // the cleanup's time; 32^3x64 with FP16 links: -5 % of the solve).
    // inner tolerance floor of a round: what an FP32 solve reliably reaches
    // (with FP16-stored links a floor of 1e-2 saved 5 % of the cleanup
    // products on the 32^3x64 lattice and no time, so one default serves both)
    const double floor_tol = p.refine_floor > 0 ? p.refine_floor : 1e-5;
    // one refinement batch: up to 16 (RHS, shift) pairs, each solving for the
    // correction of its solution from its FP64 true residual
    constexpr int CMAX = 16;
    struct Pair { int j, i; double res; };
    DMem cm;
    double2* Bm = cm.get<double2>((size_t)CMAX * n);
    double2* W = cm.get<double2>((size_t)CMAX * 2 * n);
    std::vector<Pair> pend;
    auto solve_pending = [&]() {
        const int nmem = (int)pend.size();
        if (nmem == 0) return;
        std::vector<double> tol(nmem), bnorm(nmem);
        std::vector<int> phase(nmem, 8);
        std::vector<double2> sgm(nmem);
        for (int b = 0; b < nmem; ++b) {
            const Pair& q = pend[b];
            bnorm[b] = q.res * bn[q.j];
            tol[b] = std::min(0.5, std::max(0.3 * p.tol / q.res, floor_tol));
            sgm[b] = sig[q.i];
        }
        ProjResult Rr;
        if (defl && defl->prec == GDR_PREC_F64)
            proj_run<double>(op, defl, nmem, 1, sgm, Bm, W, tol, bnorm, mc, p.max_cycles, S, phase, Rr,
                             false, 0, p.use_graph != 0);
        else
            proj_run<float>(op, defl, nmem, 1, sgm, Bm, W, tol, bnorm, mc, p.max_cycles, S, phase, Rr,
                            false, 0, p.use_graph != 0, p.sstep, p.sstep_reorth,
                            /*replace=*/false);
        for (int b = 0; b < nmem; ++b) {
            const Pair& q = pend[b];
            axpy_dev(X_eo + ((int64_t)q.j * ns + q.i) * n, 0, W + (int64_t)b * 2 * n, 0, nullptr, 0, n,
                     1, st);
            if (S.st) {
                S.st->mvp_cleanup += Rr.mvps[b];
                S.st->cycles_cleanup += Rr.cycles[b];
            }
        }
        HIPCHK(hipStreamSynchronize(st));
        pend.clear();
    };
    for (int round = 0; round <= p.max_refine && !done; ++round) {
        // Every pair's FP64 true residual, one right-hand side's shifts per
        // operator launch. A pair above tolerance takes a copy of its residual
        // into the next batch slot (the pairs are independent, so a full batch
        // is solved at once, before the later right-hand sides are checked).
        const bool solve = round < p.max_refine;
        int above = 0;
        for (int j = 0; j < nrhs; ++j) {
            residual_vectors(op, ns, sig, B_eo + (int64_t)j * n, X_eo + (int64_t)j * ns * n, R);
            auto rn = norms_of(op, R, ns);
            if (S.st) S.st->mvp_fp64 += ns;
            for (int i = 0; i < ns; ++i) {
                const double rel = bn[j] > 0 ? rn[i] / bn[j] : rn[i];
                if (!std::isfinite(rel))
                    throw GdrError(GDR_ERR_BREAKDOWN, "mixed-precision cleanup: non-finite true residual");
                if (round == 0 && S.st) S.st->resid_main = std::max(S.st->resid_main, rel);
                if (rel <= p.tol) continue;
                ++above;
                if (!solve) continue;
                copy_vec(R + (int64_t)i * n, 0, Bm + (int64_t)pend.size() * n, 0, n, 1, st);
                pend.push_back({j, i, rel});
                if ((int)pend.size() == CMAX) solve_pending();
            }
        }
        solve_pending();
        done = above == 0;
        if (!solve) break;
    }
    return done ? GDR_OK : GDR_NOT_CONVERGED;
}

}  // namespace gdr
