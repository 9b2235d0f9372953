// C entry points of libelm (declared and documented in include/elm.h):
// argument validation, workspace, stream handling and the refinement loop.
// All device work is in the kernels of the other translation units.
#include "elm_internal.h"

#include <algorithm>
#include <thread>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <new>

namespace elm {

void* Workspace::get(const std::string& name, size_t bytes) {
    if (bytes == 0) bytes = 256;
    for (auto& kv : bufs) {
        if (kv.first == name) {
            if (kv.second.bytes >= bytes) return kv.second.ptr;
            // grow: hipFree waits for pending work on the buffer
            ELM_HIP_TRY(hipFree(kv.second.ptr));
            kv.second.ptr = nullptr;
            kv.second.bytes = 0;
            void* p = nullptr;
            if (hipMalloc(&p, bytes) != hipSuccess)
                throw Error{ELM_ERR_ALLOC, "workspace '" + name + "': hipMalloc of " +
                                               std::to_string(bytes) + " bytes failed"};
            kv.second.ptr = p;
            kv.second.bytes = bytes;
            return p;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        throw Error{ELM_ERR_ALLOC,
                    "workspace '" + name + "': hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    bufs.push_back({name, Buffer{p, bytes}});
    return p;
}

void Workspace::release() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
    for (auto& kv : bufs)
        if (kv.second.ptr) (void)hipFree(kv.second.ptr);
    bufs.clear();
    tables.clear();
}

hipEvent_t Profiler::take() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    ELM_HIP_TRY(hipEventCreate(&e));
    return e;
}

void Profiler::resolve() {
    for (auto& pe : pending) {
        ELM_HIP_TRY(hipEventSynchronize(pe.b));
        float t = 0;
        ELM_HIP_TRY(hipEventElapsedTime(&t, pe.a, pe.b));
        ms[pe.stage] += t;
        cnt[pe.stage] += 1;
        pool.push_back(pe.a);
        pool.push_back(pe.b);
    }
    pending.clear();
}

void Profiler::release() {
    for (auto& pe : pending) {
        (void)hipEventDestroy(pe.a);
        (void)hipEventDestroy(pe.b);
    }
    pending.clear();
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
}

StageScope::StageScope(Profiler* prof, int st, hipStream_t stream) : p(prof), stage(st), s(stream) {
    if (p && p->on) {
        a = p->take();
        ELM_HIP_TRY(hipEventRecord(a, s));
    }
}

StageScope::~StageScope() {
    if (!a) return;
    hipEvent_t b = nullptr;
    try {
        b = p->take();
    } catch (...) {
        return;
    }
    if (hipEventRecord(b, s) == hipSuccess) p->pending.push_back({stage, a, b});
}

namespace {

elm_status fail(elm_handle* h, elm_status st, const std::string& msg) {
    if (h) h->last_error = msg;
    return st;
}

// Runs `body` and turns exceptions into status codes.  Bodies validate every
// argument first (pure host checks) and call use_device() before any HIP call.
template <typename F>
elm_status guarded(elm_handle* h, F&& body) {
    try {
        if (h) h->last_error.clear();
        body();
        return ELM_OK;
    } catch (const Error& e) {
        return fail(h, e.st, e.msg);
    } catch (const std::bad_alloc&) {
        return fail(h, ELM_ERR_ALLOC, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(h, ELM_ERR_HIP, e.what());
    }
}

void use_device(elm_handle* h) { ELM_HIP_TRY(hipSetDevice(h->device)); }

// a nested entry point's failure, rethrown with its message
void check_status(elm_handle* h, elm_status st) {
    if (st != ELM_OK) throw Error{st, h->last_error};
}

#define REQUIRE(cond, st, msg) \
    do {                       \
        if (!(cond)) throw ::elm::Error{st, msg}; \
    } while (0)

size_t dtype_size(elm_dtype dt) {
    switch (dt) {
        case ELM_F64: return 8;
        case ELM_F32: return 4;
        case ELM_BF16: return 2;
        case ELM_F16: return 2;
    }
    return 0;
}

void free_factor_buffers(elm_factor* f) {
    if (!f) return;
    if (f->pool || f->arena) {  // workspace and arena buffers stay where they are
        f->piv = nullptr;
        f->R = f->Rinv = f->K = f->Usinv = f->RinvT = f->KT = f->UsinvT = nullptr;
        return;
    }
    if (f->piv) (void)hipFree(f->piv);
    if (f->R) (void)hipFree(f->R);
    if (f->Rinv) (void)hipFree(f->Rinv);
    if (f->K) (void)hipFree(f->K);
    if (f->Usinv) (void)hipFree(f->Usinv);
    if (f->RinvT) (void)hipFree(f->RinvT);
    if (f->KT) (void)hipFree(f->KT);
    if (f->UsinvT) (void)hipFree(f->UsinvT);
    f->piv = nullptr;
    f->R = f->Rinv = f->K = f->Usinv = f->RinvT = f->KT = f->UsinvT = nullptr;
}

}  // namespace
}  // namespace elm

using elm::Error;

extern "C" {

elm_status elm_create(elm_handle** out, void* stream) {
    if (!out) return ELM_ERR_INVALID_ARG;
    *out = nullptr;
    elm_handle* h = nullptr;
    try {
        h = new elm_handle();
        h->ws.prof = &h->prof;
        h->stream = (hipStream_t)stream;
        if (hipGetDevice(&h->device) != hipSuccess) {
            delete h;
            return ELM_ERR_HIP;
        }
        int cu = 0;
        if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, h->device) == hipSuccess &&
            cu > 0)
            h->num_cu = cu;
        // set-up of elm_gram_noalloc's static scratch on this device (its
        // address is looked up once per device); a failure here is reported
        // by that entry point's first call instead
        try {
            (void)elm::noalloc_scratch(h->device);
        } catch (const elm::Error&) {
        }
    } catch (...) {
        delete h;
        return ELM_ERR_ALLOC;
    }
    *out = h;
    return ELM_OK;
}

elm_status elm_destroy(elm_handle* h) {
    if (!h) return ELM_OK;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);
    for (elm_handle* w : h->workers) elm_destroy(w);
    h->workers.clear();
    if (h->side) (void)hipStreamSynchronize(h->side);
    if (h->batch_stream) (void)hipStreamSynchronize(h->batch_stream);
    h->prof.release();
    h->ws.release();
    for (auto& e : h->side_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->batch_stream) (void)hipStreamDestroy(h->batch_stream);
    if (h->owns_stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return ELM_OK;
}

elm_status elm_set_stream(elm_handle* h, void* stream) {
    if (!h) return ELM_ERR_INVALID_ARG;
    h->stream = (hipStream_t)stream;
    return ELM_OK;
}

const char* elm_status_string(elm_status s) {
    switch (s) {
        case ELM_OK: return "ok";
        case ELM_ERR_INVALID_ARG: return "invalid argument";
        case ELM_ERR_SHAPE: return "inconsistent shape or leading dimension";
        case ELM_ERR_ALLOC: return "device allocation failed";
        case ELM_ERR_HIP: return "HIP runtime error";
        case ELM_ERR_NOT_PSD: return "Gram matrix not positive semidefinite (non-finite input)";
        case ELM_ERR_NO_CONVERGENCE: return "refinement did not reach the requested residual";
        case ELM_ERR_UNSUPPORTED: return "unsupported dtype/layout combination";
    }
    return "unknown status";
}

const char* elm_last_error(const elm_handle* h) { return h ? h->last_error.c_str() : ""; }

elm_status elm_hidden(elm_handle* h, int64_t N, int64_t d, int64_t L, const void* X, int64_t ldx,
                      const void* W, int64_t ldw, const void* b, elm_dtype dt, void* H, int64_t ldh,
                      void* Hlp, int64_t ldlp, elm_dtype lp_dt) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(N >= 1 && d >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N, d and L must be >= 1");
        REQUIRE(X && W && b, ELM_ERR_INVALID_ARG, "X, W and b must be non-null");
        REQUIRE(dt == ELM_F64 || dt == ELM_F32, ELM_ERR_UNSUPPORTED, "dt must be ELM_F64 or ELM_F32");
        REQUIRE(H || Hlp, ELM_ERR_INVALID_ARG, "at least one of H and Hlp must be non-null");
        REQUIRE(ldx >= d, ELM_ERR_SHAPE, "ldx < d");
        REQUIRE(ldw >= L, ELM_ERR_SHAPE, "ldw < L");
        if (H) REQUIRE(ldh >= L, ELM_ERR_SHAPE, "ldh < L");
        if (Hlp) {
            REQUIRE(lp_dt == ELM_BF16 || lp_dt == ELM_F16 || lp_dt == ELM_F32, ELM_ERR_UNSUPPORTED,
                    "lp_dt must be ELM_BF16, ELM_F16 or ELM_F32");
            REQUIRE(ldlp >= N, ELM_ERR_SHAPE, "ldlp < N");
        }
        elm::use_device(h);
        elm::StageScope sc(&h->prof, ELM_STAGE_HIDDEN, h->stream);
        elm::launch_hidden(h->stream, dt, N, d, L, X, ldx, W, ldw, b, H, ldh, Hlp, ldlp, lp_dt);
    });
}

}  // extern "C"

// The rank step and factor tail of a Gram M (n x n FP64, ld n, in the handle's
// workspace buffer "gram_M" or any scratch it may overwrite) already formed for
// factor f (N, L, n, transposed, gram_dtype, device and pool set); kc: products
// summed in FP32 per Gram partial (0 for an FP64 Gram).
static void factor_gram(elm_handle* h, elm_factor* f, double* M, int64_t kc, double tau_rel,
                        elm::Workspace* pool) {
    const int64_t N = f->N, L = f->L, n = f->n;
    const bool transposed = f->transposed;
    const elm_dtype h_dt = f->gram_dtype;
    // tau from the largest diagonal entry (read back once)
    double* dmax = (double*)h->ws.get("gram_dmax", sizeof(double));
    elm::launch_diag_max(h->stream, n, M, n, dmax);
    double hdmax = 0;
    ELM_HIP_TRY(hipMemcpyAsync(&hdmax, dmax, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    // an order the certified path may take: its diagonal too, in the same read
    const bool cert_order = h->full_rank_min_order > 0 && n >= h->full_rank_min_order;
    std::vector<double> hdiag;
    if (cert_order) {
        double* dg = (double*)h->ws.get("gram_diag", (size_t)n * sizeof(double));
        elm::launch_diag_copy(h->stream, n, M, n, dg);
        hdiag.resize((size_t)n);
        ELM_HIP_TRY(hipMemcpyAsync(hdiag.data(), dg, (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                                   h->stream));
    }
    ELM_HIP_TRY(hipStreamSynchronize(h->stream));
    if (!std::isfinite(hdmax)) throw Error{ELM_ERR_NOT_PSD, "Gram has a non-finite diagonal entry"};
    // default threshold: 16 (n + K) 2^-53 max diag, K = products summed per
    // Gram entry, so that the Gram's own rounding (up to K u of an entry)
    // never passes for a pivot
    const int64_t K = transposed ? L : N;
    f->tau = (tau_rel > 0 ? tau_rel : 16.0 * (double)(n + K) * std::ldexp(1.0, -53)) * hdmax;
    f->max_diag = hdmax;
    f->noise_floor = elm::schur_noise_floor(h_dt, n, N > L ? N : L, kc) * hdmax;
    bool done = false;
    if (cert_order) {
        // Duplicated nodes (bitwise-equal Gram rows) are set aside: the greedy
        // rule never pivots a copy after its original (its Schur diagonal
        // is then zero up to rounding), so on the distinct nodes it is the
        // greedy rule on their Gram, which the certificate below decides.
        std::vector<int32_t> rep;
        const int64_t ndup = elm::duplicate_nodes(h->stream, n, M, n, hdiag, h->ws, rep);
        if (ndup >= 0) {
            // certified full rank: every greedy pivot is at least
            // 1 / max_j (M^-1)_jj, read off the rows of the inverse factor
            const double need = std::max(64.0 * f->tau, 2.0 * f->noise_floor);
            if (!h->side) {  // the look-ahead stream (default priority, non-blocking)
                ELM_HIP_TRY(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
                for (auto& e : h->side_ev) ELM_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            }
            bool ok;
            {
                elm::StageScope sc(&h->prof, ELM_STAGE_RANK, h->stream);
                if (ndup == 0) {
                    ok = elm::unpivoted_cholesky(h->stream, n, M, n, need, &f->R, f, h->ws, h->side,
                                                 h->side_ev[0], h->side_ev[1]);
                } else {
                    f->piv = (int32_t*)elm::factor_alloc(f, "piv", (size_t)n * sizeof(int32_t));
                    ok = elm::dedup_cholesky(h->stream, n, M, n, rep, need, &f->R, f, h->ws, h->side,
                                             h->side_ev[0], h->side_ev[1]);
                }
            }
            if (ok) {
                const int64_t r = n - ndup;
                f->r = r;
                if (ndup == 0) {
                    f->piv = (int32_t*)elm::factor_alloc(f, "piv", (size_t)n * sizeof(int32_t));
                    elm::launch_iota(h->stream, n, f->piv);
                }
                {
                    elm::StageScope sc(&h->prof, ELM_STAGE_FACTOR, h->stream);
                    elm::build_factor_tail(h->stream, f, h->ws);
                }
                const double lam = elm::inv_max_row_sumsq(h->stream, r, f->Rinv, r, h->ws);
                if (lam >= need) {
                    f->last_pivot = lam;
                    // a copy's Schur diagonal after its original is zero
                    f->first_rejected = ndup > 0 ? 0.0 : -INFINITY;
                    f->reliable = true;
                    f->certified_full_rank = ndup > 0 ? 2 : 1;
                    done = true;
                }
            }
            if (!done) {  // not certified: the greedy rule decides
                elm::free_factor_buffers(f);
                f->r = 0;
                f->q = 0;
                f->woodbury = false;
            }
        }
    }
    if (!done) {
        f->piv = (int32_t*)elm::factor_alloc(f, "piv", (size_t)n * sizeof(int32_t));
        double pst[3];
        {
            elm::StageScope sc(&h->prof, ELM_STAGE_RANK, h->stream);
            f->r = elm::pivoted_cholesky(h->stream, n, M, n, f->tau, f->piv, &f->R, pst, h->ws, f);
        }
        f->last_pivot = pst[0];
        f->first_rejected = pst[1];
        f->reliable = (f->r == 0 || f->last_pivot >= 2.0 * f->noise_floor) &&
                      (f->r == n || f->first_rejected >= -2.0 * f->noise_floor);
        {
            // a pooled factor is solved with at once (inside elm_train), so
            // its last check can wait for the solve's first synchronisation
            elm::StageScope sc(&h->prof, ELM_STAGE_FACTOR, h->stream);
            elm::build_factor_tail(h->stream, f, h->ws, /*wait=*/pool == nullptr);
        }
    }
}

static elm_status rank_factor_impl(elm_handle* h, int64_t N, int64_t L, const void* H, int64_t ldh,
                                   elm_dtype h_dt, elm_layout layout, double tau_rel,
                                   elm_factor** out, int64_t* rank, elm::Workspace* pool) {
    if (!h) return ELM_ERR_INVALID_ARG;
    elm_factor* f = nullptr;
    elm_status st = elm::guarded(h, [&] {
        REQUIRE(out, ELM_ERR_INVALID_ARG, "out must be non-null");
        *out = nullptr;
        REQUIRE(N >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N and L must be >= 1");
        REQUIRE(H, ELM_ERR_INVALID_ARG, "H must be non-null");
        REQUIRE(tau_rel < 1.0 && !std::isnan(tau_rel), ELM_ERR_INVALID_ARG, "tau_rel must be < 1");
        REQUIRE(layout == ELM_SAMPLE_MAJOR || layout == ELM_NODE_MAJOR, ELM_ERR_INVALID_ARG,
                "unknown layout");
        REQUIRE(h_dt == ELM_F64 || h_dt == ELM_F32 || h_dt == ELM_BF16 || h_dt == ELM_F16,
                ELM_ERR_INVALID_ARG, "unknown dtype");
        REQUIRE(ldh >= (layout == ELM_SAMPLE_MAJOR ? L : N), ELM_ERR_SHAPE,
                "ldh smaller than the row length");
        const bool transposed = N < L;
        if (h_dt == ELM_F64)
            REQUIRE(layout == ELM_SAMPLE_MAJOR, ELM_ERR_UNSUPPORTED, "FP64 H must be sample-major");
        else
            REQUIRE(layout == ELM_NODE_MAJOR && !transposed, ELM_ERR_UNSUPPORTED,
                    "low-precision H must be node-major, with N >= L");
        const int64_t n = transposed ? N : L;
        elm::use_device(h);
        f = new elm_factor();
        f->N = N;
        f->L = L;
        f->n = n;
        f->transposed = transposed;
        f->device = h->device;
        f->pool = pool;
        double* M = (double*)h->ws.get("gram_M", (size_t)n * n * sizeof(double));
        int64_t kc = 0;  // products accumulated in FP32 per partial (low-precision Grams)
        if (h_dt == ELM_F64) {
            if (transposed)
                elm::launch_gram_f64_rows(h->stream, N, L, (const double*)H, ldh, M, n, h->ws);
            else
                elm::launch_gram_f64_cols(h->stream, N, L, (const double*)H, ldh, M, n, h->ws);
        } else {
            kc = elm::launch_gram_lp_nodes(h->stream, h_dt, N, L, H, ldh, M, n, h->ws);
        }
        f->gram_dtype = h_dt;
        factor_gram(h, f, M, kc, tau_rel, pool);
        if (rank) *rank = f->r;
        *out = f;
    });
    if (st != ELM_OK && f) {
        elm::free_factor_buffers(f);
        delete f;
    }
    return st;
}

extern "C" {

elm_status elm_rank_factor(elm_handle* h, int64_t N, int64_t L, const void* H, int64_t ldh,
                           elm_dtype h_dt, elm_layout layout, double tau_rel, elm_factor** out,
                           int64_t* rank) {
    return rank_factor_impl(h, N, L, H, ldh, h_dt, layout, tau_rel, out, rank, nullptr);
}

elm_status elm_factor_grow(elm_handle* h, const elm_factor* f, int64_t N, int64_t L, const double* H64,
                           int64_t ldh64, double tau_rel, elm_factor** out, int64_t* rank, int32_t* grown) {
    if (!h) return ELM_ERR_INVALID_ARG;
    elm_factor* g = nullptr;
    elm_status st = elm::guarded(h, [&] {
        REQUIRE(out, ELM_ERR_INVALID_ARG, "out must be non-null");
        *out = nullptr;
        REQUIRE(f && H64, ELM_ERR_INVALID_ARG, "f and H64 must be non-null");
        REQUIRE(tau_rel < 1.0 && !std::isnan(tau_rel), ELM_ERR_INVALID_ARG, "tau_rel must be < 1");
        REQUIRE(!f->transposed && f->gram_dtype == ELM_F64, ELM_ERR_UNSUPPORTED,
                "growth needs a factor of the FP64 column Gram H^T H");
        REQUIRE(N == f->N, ELM_ERR_SHAPE, "N differs from the factor's");
        REQUIRE(L > f->L, ELM_ERR_SHAPE, "L must exceed the factor's number of nodes");
        REQUIRE(N >= L, ELM_ERR_UNSUPPORTED, "growth keeps the column Gram: N >= L");
        REQUIRE(ldh64 >= L, ELM_ERR_SHAPE, "ldh64 < L");
        elm::use_device(h);
        g = new elm_factor();
        g->device = h->device;
        bool ok;
        {
            elm::StageScope sc(&h->prof, ELM_STAGE_RANK, h->stream);
            ok = elm::grow_factor(h->stream, f, N, L, H64, ldh64, tau_rel, g, h->ws);
        }
        if (!ok) {  // the old decision does not stand under the grown threshold
            delete g;
            g = nullptr;
            elm::check_status(h, rank_factor_impl(h, N, L, H64, ldh64, ELM_F64, ELM_SAMPLE_MAJOR, tau_rel,
                                                  &g, nullptr, nullptr));
        }
        if (grown) *grown = ok ? 1 : 0;
        if (rank) *rank = g->r;
        *out = g;
        g = nullptr;
    });
    if (g) {
        elm::free_factor_buffers(g);
        delete g;
    }
    return st;
}

elm_status elm_gram(elm_handle* h, int64_t N, int64_t L, const void* H, int64_t ldh, elm_dtype h_dt,
                    elm_layout layout, double* M, int64_t ldm) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(N >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N and L must be >= 1");
        REQUIRE(H && M, ELM_ERR_INVALID_ARG, "H and M must be non-null");
        REQUIRE(layout == ELM_SAMPLE_MAJOR || layout == ELM_NODE_MAJOR, ELM_ERR_INVALID_ARG,
                "unknown layout");
        REQUIRE(h_dt == ELM_F64 || h_dt == ELM_F32 || h_dt == ELM_BF16 || h_dt == ELM_F16,
                ELM_ERR_INVALID_ARG, "unknown dtype");
        REQUIRE(ldh >= (layout == ELM_SAMPLE_MAJOR ? L : N), ELM_ERR_SHAPE,
                "ldh smaller than the row length");
        const bool transposed = N < L;
        const int64_t n = transposed ? N : L;
        REQUIRE(ldm >= n, ELM_ERR_SHAPE, "ldm < min(N, L)");
        if (h_dt == ELM_F64)
            REQUIRE(layout == ELM_SAMPLE_MAJOR, ELM_ERR_UNSUPPORTED, "FP64 H must be sample-major");
        else
            REQUIRE(layout == ELM_NODE_MAJOR && !transposed, ELM_ERR_UNSUPPORTED,
                    "low-precision H must be node-major, with N >= L");
        elm::use_device(h);
        if (h_dt == ELM_F64) {
            if (transposed)
                elm::launch_gram_f64_rows(h->stream, N, L, (const double*)H, ldh, M, ldm, h->ws);
            else
                elm::launch_gram_f64_cols(h->stream, N, L, (const double*)H, ldh, M, ldm, h->ws);
        } else {
            elm::launch_gram_lp_nodes(h->stream, h_dt, N, L, H, ldh, M, ldm, h->ws);
        }
    });
}

elm_status elm_gram_noalloc(elm_handle* h, int64_t N, int64_t L, const void* H, int64_t ldh,
                            elm_dtype h_dt, elm_layout layout, double* M, int64_t ldm) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(N >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N and L must be >= 1");
        REQUIRE(H && M, ELM_ERR_INVALID_ARG, "H and M must be non-null");
        REQUIRE(layout == ELM_SAMPLE_MAJOR || layout == ELM_NODE_MAJOR, ELM_ERR_INVALID_ARG,
                "unknown layout");
        REQUIRE(h_dt == ELM_F64 || h_dt == ELM_F32 || h_dt == ELM_BF16 || h_dt == ELM_F16,
                ELM_ERR_INVALID_ARG, "unknown dtype");
        REQUIRE(ldh >= (layout == ELM_SAMPLE_MAJOR ? L : N), ELM_ERR_SHAPE,
                "ldh smaller than the row length");
        const bool transposed = N < L;
        const int64_t n = transposed ? N : L;
        REQUIRE(ldm >= n, ELM_ERR_SHAPE, "ldm < min(N, L)");
        if (h_dt == ELM_F64)
            REQUIRE(layout == ELM_SAMPLE_MAJOR, ELM_ERR_UNSUPPORTED, "FP64 H must be sample-major");
        else
            REQUIRE(layout == ELM_NODE_MAJOR && !transposed, ELM_ERR_UNSUPPORTED,
                    "low-precision H must be node-major, with N >= L");
        elm::use_device(h);
        elm::launch_gram_noalloc(h->stream, h->device, h_dt, N, L, H, ldh, M, ldm);
    });
}

elm_status elm_autotune_gram(elm_handle* h, int64_t N, int64_t L, const void* Hn, int64_t ldn,
                             elm_dtype dt, int32_t* splits_out, double* ms_out) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(N >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N and L must be >= 1");
        REQUIRE(Hn, ELM_ERR_INVALID_ARG, "Hn must be non-null");
        REQUIRE(dt == ELM_BF16 || dt == ELM_F16 || dt == ELM_F32 || dt == ELM_F64, ELM_ERR_INVALID_ARG,
                "unknown dtype");
        REQUIRE(N >= L, ELM_ERR_UNSUPPORTED, "the autotuner covers the column Gram: N >= L");
        REQUIRE(ldn >= (dt == ELM_F64 ? L : N), ELM_ERR_SHAPE, "leading dimension smaller than the row");
        elm::use_device(h);
        const bool lp = dt == ELM_BF16 || dt == ELM_F16;
        const int base = lp ? elm::gram_default_splits(N, L) : elm::gram16_default_chunks(dt, L, N);
        std::vector<int> cand;
        for (double f : {1.0, 0.5, 0.75, 1.5, 2.0}) {
            int c = (int)std::lround(base * f);
            c = std::max(1, std::min(lp ? 48 : 64, c));
            while (lp && c > 1 && N / c < 2048) --c;
            if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
        }
        double* M = (double*)h->ws.get("tune_M", (size_t)L * L * sizeof(double));
        auto gram = [&](int c) {
            if (dt == ELM_F64)
                elm::launch_gram_f64_cols(h->stream, N, L, (const double*)Hn, ldn, M, L, h->ws, c);
            else
                elm::launch_gram_lp_nodes(h->stream, dt, N, L, Hn, ldn, M, L, h->ws, c);
        };
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ELM_HIP_TRY(hipEventCreate(&e0));
        ELM_HIP_TRY(hipEventCreate(&e1));
        struct Ev {
            hipEvent_t a, b;
            ~Ev() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } ev{e0, e1};
        // the default rule's count stays unless another is at least 2% faster
        int best = cand[0];
        double best_ms = 1e300, base_ms = 0.0;
        for (int c : cand) {
            // one untimed run (tables, partial buffer), then the mean of two
            gram(c);
            ELM_HIP_TRY(hipEventRecord(e0, h->stream));
            for (int r = 0; r < 2; ++r) gram(c);
            ELM_HIP_TRY(hipEventRecord(e1, h->stream));
            ELM_HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            ELM_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            const double t = ms / 2.0;
            if (c == cand[0]) {
                base_ms = t;
                best_ms = t;
            } else if (t < best_ms && t < 0.98 * base_ms) {
                best_ms = t;
                best = c;
            }
        }
        h->ws.put_tune(lp ? ELM_TUNE_GRAM_SPLITS : ELM_TUNE_GRAM_CHUNKS, (int)dt, L, N, best);
        if (splits_out) *splits_out = best;
        if (ms_out) *ms_out = best_ms;
    });
}

elm_status elm_tune_table_get(const elm_handle* h, elm_tune_entry* out, int32_t capacity, int32_t* count) {
    if (!h || !count || capacity < 0 || (capacity > 0 && !out)) return ELM_ERR_INVALID_ARG;
    *count = (int32_t)h->ws.tune.size();
    for (int32_t i = 0; i < *count && i < capacity; ++i) out[i] = h->ws.tune[(size_t)i];
    return ELM_OK;
}

namespace elm {
namespace {
bool tune_row_ok(const elm_tune_entry& t) {
    if (t.kind == ELM_TUNE_PANEL) return t.value == 32 || t.value == 64 || t.value == 128 || t.value == 256;
    if (t.kind == ELM_TUNE_GRAM_SPLITS || t.kind == ELM_TUNE_GRAM_CHUNKS)
        return t.value >= 1 && t.value <= 64 && t.dtype >= ELM_F64 && t.dtype <= ELM_F16;
    return false;
}
}  // namespace
}  // namespace elm

elm_status elm_tune_table_set(elm_handle* h, const elm_tune_entry* rows, int32_t count) {
    if (!h || count < 0 || (count > 0 && !rows)) return ELM_ERR_INVALID_ARG;
    for (int32_t i = 0; i < count; ++i)
        if (!elm::tune_row_ok(rows[i])) return ELM_ERR_INVALID_ARG;
    h->ws.tune.assign(rows, rows + count);
    return ELM_OK;
}

elm_status elm_tune_table_save(const elm_handle* h, const char* path) {
    if (!h || !path) return ELM_ERR_INVALID_ARG;
    FILE* fp = std::fopen(path, "w");
    if (!fp) return ELM_ERR_INVALID_ARG;
    std::fprintf(fp, "# libelm tuning table: kind dtype n_log2 k_log2 value\n");
    for (const elm_tune_entry& t : h->ws.tune)
        std::fprintf(fp, "%d %d %d %d %d\n", t.kind, t.dtype, t.n_log2, t.k_log2, t.value);
    const bool ok = std::fclose(fp) == 0;
    return ok ? ELM_OK : ELM_ERR_INVALID_ARG;
}

elm_status elm_tune_table_load(elm_handle* h, const char* path) {
    if (!h || !path) return ELM_ERR_INVALID_ARG;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return ELM_ERR_INVALID_ARG;
    std::vector<elm_tune_entry> rows;
    char line[256];
    bool ok = true;
    while (std::fgets(line, sizeof(line), fp)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        elm_tune_entry t{};
        if (std::sscanf(line, "%d %d %d %d %d", &t.kind, &t.dtype, &t.n_log2, &t.k_log2, &t.value) != 5 ||
            !elm::tune_row_ok(t)) {
            ok = false;
            break;
        }
        rows.push_back(t);
    }
    std::fclose(fp);
    if (!ok) return ELM_ERR_INVALID_ARG;
    h->ws.tune = rows;
    return ELM_OK;
}

elm_status elm_factor_rank(const elm_factor* f, int64_t* rank) {
    if (!f || !rank) return ELM_ERR_INVALID_ARG;
    *rank = f->r;
    return ELM_OK;
}

elm_status elm_factor_get_info(const elm_factor* f, elm_factor_info* out) {
    if (!f || !out) return ELM_ERR_INVALID_ARG;
    out->rank = f->r;
    out->n = f->n;
    out->transposed = f->transposed ? 1 : 0;
    out->gram_dtype = (int32_t)f->gram_dtype;
    out->max_diag = f->max_diag;
    out->last_pivot = f->last_pivot;
    out->first_rejected = f->first_rejected;
    out->tau = f->tau;
    out->noise_floor = f->noise_floor;
    out->reliable = f->reliable ? 1 : 0;
    out->certified_full_rank = f->certified_full_rank;
    return ELM_OK;
}

elm_status elm_factor_pivots(elm_handle* h, const elm_factor* f, int32_t* piv_host) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(f && piv_host, ELM_ERR_INVALID_ARG, "factor and piv_host must be non-null");
        elm::use_device(h);
        ELM_HIP_TRY(hipMemcpyAsync(piv_host, f->piv, (size_t)f->n * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, h->stream));
        ELM_HIP_TRY(hipStreamSynchronize(h->stream));
    });
}

elm_status elm_factor_destroy(elm_factor* f) {
    if (!f) return ELM_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(f->device);
    (void)hipDeviceSynchronize();
    elm::free_factor_buffers(f);
    (void)hipSetDevice(cur);
    delete f;
    return ELM_OK;
}

}  // extern "C"

namespace elm {
namespace {

// beta = H^+ T with refinement (see elm_pinv_solve).  With z_ready the
// caller has already put Z = H^T T and ||Z||_F^2 in the workspace buffers
// "ps_Z" / "ps_nrm" (the hidden-layer kernel can produce them on the fly).
// Y / labels (optional): H beta and its row arg-max for the returned beta,
// taken from the last residual pass (a separate pass when there is none).
elm_status pinv_solve_impl(elm_handle* h, const elm_factor* f, int64_t m, const double* T, int64_t ldt,
                           const double* H64, int64_t ldh64, double ir_tol, int32_t ir_max_iter,
                           double* beta, int64_t ldbeta, elm_solve_info* info, bool z_ready,
                           double* Y = nullptr, int64_t ldy = 0, int32_t* labels = nullptr) {
    elm_status result = ELM_OK;
    const int64_t N = f->N, L = f->L;
    elm::use_device(h);
    hipStream_t s = h->stream;
    elm::Workspace& ws = h->ws;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->rank = f->r;
        info->transposed = f->transposed ? 1 : 0;
        info->ne_residual = -1.0;
    }
    double* Z = (double*)ws.get("ps_Z", (size_t)L * m * sizeof(double));
    double* nrm = (double*)ws.get("ps_nrm", 2 * sizeof(double));
    // beta_0 = H^+ T
    elm::Profiler* pr = &h->prof;
    if (!f->transposed) {
        if (!z_ready) {
            elm::StageScope sc(pr, ELM_STAGE_RHS, s);
            elm::launch_ht_times(s, N, L, m, H64, ldh64, T, ldt, Z, m, nrm, ws);   // H^T T, eq. (8)
        }
        elm::StageScope sc(pr, ELM_STAGE_SOLVE, s);
        elm::apply_pinv(s, f, m, Z, m, H64, ldh64, beta, ldbeta, ws);
    } else {
        elm::StageScope sc(pr, ELM_STAGE_SOLVE, s);
        elm::apply_pinv(s, f, m, T, ldt, H64, ldh64, beta, ldbeta, ws);
    }
    // a factor built without waiting: its Gram-of-G flag is read at the
    // first synchronisation below
    int pd_bad = 0;
    if (f->pd_flag)
        ELM_HIP_TRY(hipMemcpyAsync(&pd_bad, f->pd_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    auto check_pd = [&] {
        if (pd_bad) throw elm::Error{ELM_ERR_NOT_PSD, "Gram of G is not positive definite"};
    };
    if (ir_max_iter == 0) {
        if (Y || labels) {
            elm::StageScope sc(pr, ELM_STAGE_PREDICT, s);
            elm::launch_hidden_output(s, N, L, m, H64, ldh64, beta, ldbeta, Y, ldy, labels);
        }
        ELM_HIP_TRY(hipStreamSynchronize(s));
        check_pd();
        return result;
    }
    if (f->transposed && !z_ready) {
        elm::StageScope sc(pr, ELM_STAGE_RHS, s);
        elm::launch_ht_times(s, N, L, m, H64, ldh64, T, ldt, Z, m, nrm, ws);
    }
    double* E = (double*)ws.get("ps_E", (size_t)N * m * sizeof(double));
    double* G = (double*)ws.get("ps_G", (size_t)L * m * sizeof(double));
    double* D = (double*)ws.get("ps_D", (size_t)L * m * sizeof(double));
    double* Bprev = (double*)ws.get("ps_Bprev", (size_t)L * m * sizeof(double));
    // the loop's decisions are taken on the device by the kernel the batched
    // refinement uses (so a batch and a single training decide alike); the
    // host reads the state back once per iteration
    elm::RefineDesc one;
    one.g2 = nrm + 1;
    one.z2 = nrm;
    elm::RefineDesc* done_d = (elm::RefineDesc*)ws.get("ps_desc", sizeof(elm::RefineDesc));
    elm::IrCtl* ctl = (elm::IrCtl*)ws.get("ps_ctl", sizeof(elm::IrCtl));
    int32_t* flags = (int32_t*)ws.get("ps_flags", 3 * sizeof(int32_t));
    ELM_HIP_TRY(hipMemcpyAsync(done_d, &one, sizeof(one), hipMemcpyHostToDevice, s));
    elm::launch_ir_init(s, 1, ctl, flags, flags + 1);
    elm::IrCtl hc;
    int32_t hflags[2] = {0, 0};
    for (;;) {
        // G = H^T (T - H beta): two streaming passes over H
        {
            elm::StageScope sc(pr, ELM_STAGE_RESIDUAL, s);
            elm::launch_residual(s, N, L, m, H64, ldh64, T, ldt, beta, ldbeta, E, m, Y, ldy, labels);
        }
        {
            elm::StageScope sc(pr, ELM_STAGE_RHS, s);
            elm::launch_ht_times(s, N, L, m, H64, ldh64, E, m, G, m, nrm + 1, ws);
        }
        elm::launch_ir_decide(s, 1, ctl, done_d, flags, flags + 1, flags + 2, ir_tol, ir_max_iter);
        ELM_HIP_TRY(hipMemcpyAsync(&hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, s));
        ELM_HIP_TRY(hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
        ELM_HIP_TRY(hipStreamSynchronize(s));
        check_pd();
        if (hflags[1]) {
            // a diverging correction is taken back: beta is the previous iterate
            ELM_HIP_TRY(hipMemcpy2DAsync(beta, (size_t)ldbeta * sizeof(double), Bprev,
                                         (size_t)m * sizeof(double), (size_t)m * sizeof(double),
                                         (size_t)L, hipMemcpyDeviceToDevice, s));
            if (Y || labels) {
                elm::StageScope sc(pr, ELM_STAGE_PREDICT, s);
                elm::launch_hidden_output(s, N, L, m, H64, ldh64, beta, ldbeta, Y, ldy, labels);
            }
        }
        if (!hc.active) break;
        {
            elm::StageScope sc(pr, ELM_STAGE_SOLVE, s);
            if (!f->transposed)
                elm::apply_pinv(s, f, m, G, m, H64, ldh64, D, m, ws);
            else
                elm::apply_pinv(s, f, m, E, m, H64, ldh64, D, m, ws);
        }
        elm::launch_axpy_mat(s, L, m, D, m, beta, ldbeta, Bprev);
    }
    const double res = hc.res;
    const int it = hc.it;
    if (info) {
        info->iterations = it;
        info->ne_residual = res;
        for (int k = 0; k < 32; ++k) info->ne_history[k] = hc.hist[k];
    }
    if (res > ir_tol) {
        result = ELM_ERR_NO_CONVERGENCE;
        char msg[160];
        std::snprintf(msg, sizeof(msg),
                      "refinement stopped after %d iterations at relative normal-equation "
                      "residual %.3e > ir_tol %.3e",
                      it, res, ir_tol);
        h->last_error = msg;
    }
    return result;
}

// One problem of a batch refined by refine_grouped.
struct GroupedSolve {
    const elm_factor* f = nullptr;  // non-transposed, rank >= 1, checks done
    int64_t m = 0;                  // 1..16
    const double* H64 = nullptr;
    int64_t ldh64 = 0;
    const double* T = nullptr;
    int64_t ldt = 0;
    double* beta = nullptr;
    int64_t ldbeta = 0;
    const double* Z = nullptr;  // H^T T (L x m, ld m)
    const double* z2 = nullptr; // ||Z||_F^2 (device)
    elm_solve_info* info = nullptr;
    elm_status status = ELM_OK;  // out: OK or NO_CONVERGENCE (message in msg)
    std::string msg;
};

// beta = H^+ T with refinement for every problem of gs: the steps, kernels,
// arithmetic and stopping rules of pinv_solve_impl for each problem, with each
// step one launch for all problems.  The loop is decided on the device (the
// kernel pinv_solve_impl uses, for every problem at once); the blocks of a
// problem that has stopped return at once, so the host issues a fixed
// sequence -- ir_max_iter + 1 residual evaluations -- which is captured once
// as a HIP graph and replayed, and reads every problem's state back once at
// the end.
void refine_grouped(elm_handle* h, hipStream_t s, std::vector<GroupedSolve>& gs, double ir_tol,
                    int32_t ir_max_iter) {
    const int P = (int)gs.size();
    if (P == 0) return;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    int maxm = 1;
    for (const GroupedSolve& g : gs) {
        if (g.f->transposed || g.f->r < 1 || g.m < 1 || g.m > 16)
            throw Error{ELM_ERR_UNSUPPORTED, "grouped refinement: unsupported problem"};
        maxm = std::max<int>(maxm, (int)g.m);
    }
    // per-problem buffers from one arena: g2 of every problem first, then
    // E, part, G, sq, D, u, t, w, t2, bd, prev of each
    auto carve = [&](char* base, std::vector<RefineDesc>* rd, std::vector<double*>* scratch) {
        size_t off = al((size_t)P * sizeof(double));
        for (int j = 0; j < P; ++j) {
            const GroupedSolve& g = gs[j];
            const elm_factor* f = g.f;
            const int64_t N = f->N, L = f->L, m = g.m, r = f->r, c = f->n - f->r;
            const size_t sz[11] = {(size_t)(N * m), refine_part_doubles(N, L, m), (size_t)(L * m),
                                   refine_sq_doubles(L, m), (size_t)(L * m), (size_t)(r * m),
                                   (size_t)(r * m), (size_t)(c * m), (size_t)(f->q * m),
                                   (size_t)(c * m), (size_t)(L * m)};
            double* ptr[11];
            for (int k = 0; k < 11; ++k) {
                ptr[k] = base ? (double*)(base + off) : nullptr;
                off += al(std::max<size_t>(sz[k], 1) * sizeof(double));
            }
            if (rd) {
                RefineDesc& q = (*rd)[j];
                q.N = N;
                q.L = L;
                q.m = (int)m;
                q.H = g.H64;
                q.ldh = g.ldh64;
                q.T = g.T;
                q.ldt = g.ldt;
                q.beta = g.beta;
                q.ldbeta = g.ldbeta;
                q.E = ptr[0];
                q.part = ptr[1];
                q.G = ptr[2];
                q.sq = ptr[3];
                q.g2 = (double*)base + j;
                q.D = ptr[4];
                q.prev = ptr[10];
                q.z2 = g.z2;
                for (int k = 0; k < 5; ++k) (*scratch)[(size_t)j * 5 + k] = ptr[5 + k];
            }
        }
        return off;
    };
    char* arena = (char*)h->ws.get("bt_refine", carve(nullptr, nullptr, nullptr));
    std::vector<RefineDesc> rd(P);
    std::vector<double*> scr((size_t)P * 5);
    carve(arena, &rd, &scr);
    const double* g2dev = (const double*)arena;
    // the apply's descriptors: row copies (0 gather Z, 1 gather G, 2 scatter u
    // into beta, 3 into D, 4 scatter K^T u into beta, 5 into D) and its seven
    // products
    std::vector<CopyRowsDesc> cp((size_t)6 * P);
    std::vector<RowprodDesc> rp((size_t)7 * P);
    for (int j = 0; j < P; ++j) {
        const GroupedSolve& g = gs[j];
        const elm_factor* f = g.f;
        const int64_t r = f->r, c = f->n - f->r, q = f->q, m = g.m;
        double *u = scr[(size_t)j * 5], *t = scr[(size_t)j * 5 + 1], *w = scr[(size_t)j * 5 + 2],
               *t2 = scr[(size_t)j * 5 + 3], *bd = scr[(size_t)j * 5 + 4];
        auto copy = [&](int k, int64_t rows, const double* src, int64_t lds, const int32_t* idx,
                        double* dst, int64_t ldd) {
            CopyRowsDesc& x = cp[(size_t)k * P + j];
            x.rows = rows;
            x.cols = m;
            x.src = src;
            x.lds = lds;
            x.idx = idx;
            x.dst = dst;
            x.ldd = ldd;
        };
        copy(0, r, g.Z, m, f->piv, u, m);                         // F^T (.) = rows piv[:r]
        copy(1, r, rd[j].G, m, f->piv, u, m);
        copy(2, r, u, m, f->piv, g.beta, g.ldbeta);               // out[piv[:r]] = u
        copy(3, r, u, m, f->piv, rd[j].D, m);
        copy(4, c, bd, m, f->piv + r, g.beta, g.ldbeta);         // out[piv[r:]] = K^T u
        copy(5, c, bd, m, f->piv + r, rd[j].D, m);
        auto prod = [&](int k, int64_t M, int64_t K, double alpha, const double* A, int64_t lda,
                        int tri, const double* B, double beta, double* C) {
            RowprodDesc& x = rp[(size_t)k * P + j];
            x.M = M;
            x.K = K;
            x.m = (int)m;
            x.tri = tri;
            x.alpha = alpha;
            x.beta = beta;
            x.A = A;
            x.lda = lda;
            x.B = B;
            x.ldb = m;
            x.C = C;
            x.ldc = m;
        };
        // (F^T F)^-1 = Rinv Rinv^T
        prod(0, r, r, 1.0, f->RinvT, r, 2, u, 0.0, t);
        prod(1, r, r, 1.0, f->Rinv, r, 1, t, 0.0, u);
        // (G G^T)^-1: Woodbury through K^T K, or S^-1 directly
        double* x = f->woodbury ? w : u;
        if (q > 0) {
            if (f->woodbury) prod(2, c, r, 1.0, f->KT, r, 0, u, 0.0, w);
            prod(3, q, q, 1.0, f->UsinvT, q, 2, x, 0.0, t2);
            prod(4, q, q, 1.0, f->Usinv, q, 1, t2, 0.0, x);
            if (f->woodbury) prod(5, r, c, -1.0, f->K, c, 0, w, 1.0, u);
        }
        if (c > 0) prod(6, c, r, 1.0, f->KT, r, 0, u, 0.0, bd);
    }
    const size_t o_cp = al((size_t)P * sizeof(RefineDesc));
    const size_t o_rp = o_cp + al(cp.size() * sizeof(CopyRowsDesc));
    const size_t dbytes = o_rp + rp.size() * sizeof(RowprodDesc);
    std::vector<char> blob(dbytes);
    std::memcpy(blob.data(), rd.data(), (size_t)P * sizeof(RefineDesc));
    std::memcpy(blob.data() + o_cp, cp.data(), cp.size() * sizeof(CopyRowsDesc));
    std::memcpy(blob.data() + o_rp, rp.data(), rp.size() * sizeof(RowprodDesc));
    char* ddesc = (char*)h->ws.get("bt_refine_desc", dbytes);
    ELM_HIP_TRY(hipMemcpyAsync(ddesc, blob.data(), dbytes, hipMemcpyHostToDevice, s));
    const RefineDesc* drd = (const RefineDesc*)ddesc;
    const CopyRowsDesc* dcp = (const CopyRowsDesc*)(ddesc + o_cp);
    const RowprodDesc* drp = (const RowprodDesc*)(ddesc + o_rp);

    // block counts of every launch kind, and the schedules of the problems
    // still iterating
    enum { K_ROWS, K_COLS, K_HTR, K_SUM, K_AXPY, K_GAT, K_SCU, K_SCB, K_P0, NK = K_P0 + 7 };
    std::vector<int64_t> nblk((size_t)NK * P, 0);
    for (int j = 0; j < P; ++j) {
        nblk[(size_t)K_ROWS * P + j] = refine_group_blocks(RefinePass::ROWS_DOT, rd[j], maxm);
        nblk[(size_t)K_COLS * P + j] = refine_group_blocks(RefinePass::COLS_DOT, rd[j], maxm);
        nblk[(size_t)K_HTR * P + j] = refine_group_blocks(RefinePass::HT_REDUCE, rd[j], maxm);
        nblk[(size_t)K_SUM * P + j] = refine_group_blocks(RefinePass::SUM, rd[j], maxm);
        nblk[(size_t)K_AXPY * P + j] = refine_group_blocks(RefinePass::AXPY, rd[j], maxm);
        nblk[(size_t)K_GAT * P + j] = copy_rows_group_blocks(cp[j]);
        nblk[(size_t)K_SCU * P + j] = copy_rows_group_blocks(cp[(size_t)2 * P + j]);
        nblk[(size_t)K_SCB * P + j] = copy_rows_group_blocks(cp[(size_t)4 * P + j]);
        for (int k = 0; k < 7; ++k)
            nblk[(size_t)(K_P0 + k) * P + j] = rowprod_group_blocks(rp[(size_t)k * P + j], maxm);
    }
    const size_t per = (size_t)2 * P + 1;
    std::vector<int32_t> hs((size_t)NK * per);
    int32_t* ds = (int32_t*)h->ws.get("bt_refine_sched", hs.size() * sizeof(int32_t));
    GroupSched sched[NK];
    // every problem in every launch; the device flags gate them
    {
        for (int k = 0; k < NK; ++k) {
            int32_t* st = hs.data() + (size_t)k * per;
            int32_t* pr_ = st + P + 1;
            int cnt = 0;
            int64_t tot = 0;
            for (int j = 0; j < P; ++j) {
                const int64_t nb = nblk[(size_t)k * P + j];
                if (nb == 0) continue;
                st[cnt] = (int32_t)tot;
                pr_[cnt] = j;
                ++cnt;
                tot += nb;
                if (tot >= INT32_MAX) throw Error{ELM_ERR_UNSUPPORTED, "grouped launch too large"};
            }
            st[cnt] = (int32_t)tot;
            sched[k].start = ds + (size_t)k * per;
            sched[k].prob = ds + (size_t)k * per + P + 1;
            sched[k].count = cnt;
            sched[k].blocks = tot;
        }
        ELM_HIP_TRY(hipMemcpyAsync(ds, hs.data(), hs.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    IrCtl* ctl = (IrCtl*)h->ws.get("bt_ir_ctl", (size_t)P * sizeof(IrCtl));
    int32_t* flags = (int32_t*)h->ws.get("bt_ir_flags", (size_t)(2 * P + 1) * sizeof(int32_t));
    int32_t* f_active = flags;
    int32_t* f_rollback = flags + P;
    int32_t* f_any = flags + 2 * P;
    auto gated = [&](int k, const int32_t* live) {
        GroupSched g = sched[k];
        g.live = live;
        return g;
    };
    // out = H^+ (.) through each factor: from Z into beta (first) or from G into D
    auto apply = [&](bool first, const int32_t* live) {
        launch_copy_rows_grouped(s, false, dcp + (first ? 0 : 1) * P, gated(K_GAT, live));
        for (int k = 0; k < 6; ++k)
            launch_rowprod_grouped(s, drp + (size_t)k * P, gated(K_P0 + k, live), maxm);
        launch_copy_rows_grouped(s, true, dcp + (size_t)(first ? 2 : 3) * P, gated(K_SCU, live));
        launch_rowprod_grouped(s, drp + (size_t)6 * P, gated(K_P0 + 6, live), maxm);
        launch_copy_rows_grouped(s, true, dcp + (size_t)(first ? 4 : 5) * P, gated(K_SCB, live));
    };
    Profiler* pr = &h->prof;
    for (GroupedSolve& g : gs) {
        g.status = ELM_OK;
        if (g.info) {
            std::memset(g.info, 0, sizeof(*g.info));
            g.info->rank = g.f->r;
            g.info->ne_residual = -1.0;
        }
    }
    // The solve as fixed launch sequences: beta_0 and iterations [k0, k1) of
    // the loop (iteration k: residual k, the decision, a taken-back
    // correction, and the next correction unless k = ir_max_iter).  With timed
    // stages when the handle profiles (launched directly then), else each
    // sequence captured once as a HIP graph and replayed.
    auto seq = [&](bool timed, bool first, int k0, int k1) {
        if (first) {
            StageScope sc(timed ? pr : nullptr, ELM_STAGE_SOLVE, s);
            apply(true, nullptr);  // beta_0 = H^+ T
            if (ir_max_iter > 0) launch_ir_init(s, P, ctl, f_active, f_rollback);
        }
        for (int k = k0; k < k1; ++k) {
            {
                StageScope sc(timed ? pr : nullptr, ELM_STAGE_RESIDUAL, s);
                launch_refine_grouped(s, RefinePass::ROWS_DOT, drd, gated(K_ROWS, f_active), maxm);
            }
            {
                StageScope sc(timed ? pr : nullptr, ELM_STAGE_RHS, s);
                launch_refine_grouped(s, RefinePass::COLS_DOT, drd, gated(K_COLS, f_active), maxm);
                launch_refine_grouped(s, RefinePass::HT_REDUCE, drd, gated(K_HTR, f_active), maxm);
                launch_refine_grouped(s, RefinePass::SUM, drd, gated(K_SUM, f_active), maxm);
            }
            launch_ir_decide(s, P, ctl, drd, f_active, f_rollback, f_any, ir_tol, ir_max_iter);
            launch_restore_grouped(s, drd, gated(K_AXPY, f_rollback));
            if (k == ir_max_iter) break;
            {
                StageScope sc(timed ? pr : nullptr, ELM_STAGE_SOLVE, s);
                apply(false, f_active);
            }
            launch_refine_grouped(s, RefinePass::AXPY, drd, gated(K_AXPY, f_active), maxm);
        }
    };
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool can_graph = !pr->on && s != nullptr && hipStreamIsCapturing(s, &cap) == hipSuccess &&
                           cap == hipStreamCaptureStatusNone;
    // the sequences depend on the descriptor and schedule addresses, the
    // problem count, every launch's block count, maxm and the loop bounds
    uint64_t hsh = 1469598103934665603ull;
    for (int64_t v : nblk) hsh = (hsh ^ (uint64_t)v) * 1099511628211ull;
    char shape[200];
    std::snprintf(shape, sizeof(shape), "refine:%p:%p:%p:%p:%d:%d:%d:%a:%llx", (const void*)ddesc,
                  (const void*)ds, (const void*)ctl, (const void*)flags, P, maxm, (int)ir_max_iter, ir_tol,
                  (unsigned long long)hsh);
    auto run_seq = [&](bool first, int k0, int k1) {
        if (!can_graph) {
            seq(pr->on, first, k0, k1);
            return;
        }
        char key[260];
        std::snprintf(key, sizeof(key), "%s:%d:%d:%d", shape, first ? 1 : 0, k0, k1);
        hipGraphExec_t exec = h->ws.find_graph(key);
        if (!exec) {
            ELM_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipGraph_t graph = nullptr;
            try {
                seq(false, first, k0, k1);
            } catch (...) {
                (void)hipStreamEndCapture(s, &graph);
                if (graph) (void)hipGraphDestroy(graph);
                throw;
            }
            ELM_HIP_TRY(hipStreamEndCapture(s, &graph));
            const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) throw Error{ELM_ERR_HIP, "graph instantiation of the refinement failed"};
            h->ws.put_graph(key, exec);
            ++h->ws.graph_captures;
        }
        ELM_HIP_TRY(hipGraphLaunch(exec, s));
        ++h->ws.graph_launches;
    };
    // The first sequence runs as many iterations as the last call of this
    // shape needed (all of them when unknown, at most ir_max_iter + 1); while
    // a problem still iterates after it, four more at a time.  Each check is
    // the read-back of every problem's state, so a repeated batch ends with
    // one.
    std::vector<IrCtl> hc(P);
    int32_t hany = 0;
    const int kmax = ir_max_iter + 1;
    int k0 = 0;
    int k1 = ir_max_iter == 0 ? 0 : std::min(kmax, std::max(1, h->ws.find_iters(shape)));
    bool first = true;
    for (;;) {
        run_seq(first, k0, k1);
        first = false;
        if (ir_max_iter > 0) {
            ELM_HIP_TRY(hipMemcpyAsync(hc.data(), ctl, (size_t)P * sizeof(IrCtl), hipMemcpyDeviceToHost, s));
            ELM_HIP_TRY(hipMemcpyAsync(&hany, f_any, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        }
        ELM_HIP_TRY(hipStreamSynchronize(s));
        ++h->ws.host_syncs;
        if (ir_max_iter == 0 || !hany || k1 >= kmax) break;
        k0 = k1;
        k1 = std::min(kmax, k1 + 4);
    }
    if (ir_max_iter > 0) {
        int need = 1;
        for (const IrCtl& c : hc) need = std::max(need, (int)c.evals);
        h->ws.put_iters(shape, need);
    }
    if (ir_max_iter == 0) return;
    for (int j = 0; j < P; ++j) {
        GroupedSolve& g = gs[j];
        const IrCtl& c = hc[j];
        if (g.info) {
            g.info->iterations = c.it;
            g.info->ne_residual = c.res;
            for (int k = 0; k < 32; ++k) g.info->ne_history[k] = c.hist[k];
        }
        if (c.res > ir_tol) {
            g.status = ELM_ERR_NO_CONVERGENCE;
            char msg[160];
            std::snprintf(msg, sizeof(msg),
                          "refinement stopped after %d iterations at relative normal-equation "
                          "residual %.3e > ir_tol %.3e",
                          c.it, c.res, ir_tol);
            g.msg = msg;
        }
    }
}

}  // namespace
}  // namespace elm

extern "C" {

elm_status elm_pinv_solve(elm_handle* h, const elm_factor* f, int64_t m, const double* T, int64_t ldt,
                          const double* H64, int64_t ldh64, double ir_tol, int32_t ir_max_iter,
                          double* beta, int64_t ldbeta, elm_solve_info* info) {
    if (!h) return ELM_ERR_INVALID_ARG;
    elm_status result = ELM_OK;
    elm_status st = elm::guarded(h, [&] {
        REQUIRE(f, ELM_ERR_INVALID_ARG, "factor must be non-null");
        REQUIRE(m >= 1 && m <= 64, ELM_ERR_INVALID_ARG, "m must be in [1, 64]");
        REQUIRE(T && H64 && beta, ELM_ERR_INVALID_ARG, "T, H64 and beta must be non-null");
        REQUIRE(ldt >= m && ldbeta >= m, ELM_ERR_SHAPE, "ldt or ldbeta smaller than m");
        REQUIRE(ldh64 >= f->L, ELM_ERR_SHAPE, "ldh64 < L");
        REQUIRE(ir_tol >= 0.0 && ir_tol < 1.0, ELM_ERR_INVALID_ARG, "ir_tol must be in [0, 1)");
        REQUIRE(ir_max_iter >= 0 && ir_max_iter <= 31, ELM_ERR_INVALID_ARG,
                "ir_max_iter must be in [0, 31]");
        result = elm::pinv_solve_impl(h, f, m, T, ldt, H64, ldh64, ir_tol, ir_max_iter, beta, ldbeta,
                                      info, false);
    });
    if (st != ELM_OK) return st;
    if (result != ELM_OK) h->last_error = "refinement stopped above ir_tol";
    return result;
}

elm_status elm_block_solve(elm_handle* h, int64_t N, int64_t L, int64_t m, const double* H64,
                           int64_t ldh64, const double* T, int64_t ldt, const double* M, int64_t ldm,
                           int64_t split, const int32_t* piv, double* beta, int64_t ldbeta) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(N >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N and L must be >= 1");
        REQUIRE(m >= 1 && m <= 64, ELM_ERR_INVALID_ARG, "m must be in [1, 64]");
        REQUIRE(H64 && T && beta, ELM_ERR_INVALID_ARG, "H64, T and beta must be non-null");
        REQUIRE(split >= 1 && split <= L, ELM_ERR_INVALID_ARG, "split must be in [1, L]");
        REQUIRE(N >= L, ELM_ERR_SHAPE, "the block form needs full column rank, so N >= L");
        REQUIRE(ldh64 >= L && ldt >= m && ldbeta >= m, ELM_ERR_SHAPE,
                "a leading dimension is smaller than its row length");
        REQUIRE(!M || ldm >= L, ELM_ERR_SHAPE, "ldm < L");
        elm::use_device(h);
        hipStream_t s = h->stream;
        // Z = H^T T (the same pass as the solves' right-hand sides)
        double* Z = (double*)h->ws.get("bs_Z", (size_t)L * m * sizeof(double));
        double* nrm = (double*)h->ws.get("bs_nrm", sizeof(double));
        {
            elm::StageScope sc(&h->prof, ELM_STAGE_RHS, s);
            elm::launch_ht_times(s, N, L, m, H64, ldh64, T, ldt, Z, m, nrm, h->ws);
        }
        if (!M) {
            double* Mw = (double*)h->ws.get("bs_M", (size_t)L * L * sizeof(double));
            elm::launch_gram_f64_cols(s, N, L, H64, ldh64, Mw, L, h->ws);
            M = Mw;
            ldm = L;
        }
        // the rank step's default threshold: a pivot of A or D at or below
        // 16 (L + N) 2^-53 max_j M_jj is a numerically dependent column
        double* dmax = (double*)h->ws.get("bs_dmax", sizeof(double));
        elm::launch_diag_max(s, L, M, ldm, dmax);
        double hmax = 0.0;
        ELM_HIP_TRY(hipMemcpyAsync(&hmax, dmax, sizeof(double), hipMemcpyDeviceToHost, s));
        ELM_HIP_TRY(hipStreamSynchronize(s));
        REQUIRE(std::isfinite(hmax), ELM_ERR_NOT_PSD, "the Gram has a non-finite diagonal");
        const double thr = 16.0 * (double)(L + N) * std::ldexp(1.0, -53) * hmax;
        elm::StageScope sc(&h->prof, ELM_STAGE_SOLVE, s);
        elm::block_solve(s, L, m, split, M, ldm, Z, m, piv, thr, beta, ldbeta, h->ws);
    });
}

}  // extern "C"

namespace elm {
namespace {

// Precision ladder of the precision form: after a failed guard the Gram is
// formed again one step up (16-bit -> FP32 -> FP64).
elm_dtype next_gram_dtype(elm_dtype dt) { return dt == ELM_F32 ? ELM_F64 : ELM_F32; }


}  // namespace
}  // namespace elm

extern "C" {

elm_status elm_train(elm_handle* h, int64_t N, int64_t d, int64_t L, int64_t m, const double* X,
                     int64_t ldx, const double* W, int64_t ldw, const double* b, const double* T,
                     int64_t ldt, elm_dtype gram_dt, double* H64, int64_t ldh64, void* Hlp,
                     int64_t ldlp, double tau_rel, double ir_tol, int32_t ir_max_iter, double* beta,
                     int64_t ldbeta, double* Y, int64_t ldy, int32_t* labels, elm_train_info* info,
                     elm_factor** factor_out) {
    if (!h) return ELM_ERR_INVALID_ARG;
    elm_factor* f = nullptr;
    elm_status st = elm::guarded(h, [&] {
        REQUIRE(N >= 1 && d >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N, d and L must be >= 1");
        REQUIRE(m >= 1 && m <= 64, ELM_ERR_INVALID_ARG, "m must be in [1, 64]");
        REQUIRE(X && W && b && T && H64 && beta, ELM_ERR_INVALID_ARG,
                "X, W, b, T, H64 and beta must be non-null");
        REQUIRE(gram_dt == ELM_F64 || gram_dt == ELM_F32 || gram_dt == ELM_BF16 || gram_dt == ELM_F16,
                ELM_ERR_INVALID_ARG, "unknown gram dtype");
        REQUIRE(ldx >= d && ldw >= L && ldt >= m && ldh64 >= L && ldbeta >= m, ELM_ERR_SHAPE,
                "a leading dimension is smaller than its row length");
        REQUIRE(!Hlp || ldlp >= N, ELM_ERR_SHAPE, "ldlp < N");
        REQUIRE(!Y || ldy >= m, ELM_ERR_SHAPE, "ldy < m");
        REQUIRE(!(Y || labels) || m <= 16, ELM_ERR_UNSUPPORTED, "training outputs need m <= 16");
        REQUIRE(ir_tol >= 0.0 && ir_tol < 1.0, ELM_ERR_INVALID_ARG, "ir_tol must be in [0, 1)");
        REQUIRE(ir_max_iter >= 0 && ir_max_iter <= 31, ELM_ERR_INVALID_ARG,
                "ir_max_iter must be in [0, 31]");
        if (factor_out) *factor_out = nullptr;
        elm::use_device(h);
        elm_train_info ti;
        std::memset(&ti, 0, sizeof(ti));
        // the low-precision Gram is formed from a node-major copy, N >= L only
        elm_dtype gdt = N < L ? ELM_F64 : gram_dt;
        const bool own_lp = gdt != ELM_F64 && !Hlp;
        void* lp = Hlp;
        int64_t ldl = ldlp;
        if (own_lp) {
            ldl = elm::lp_ld(N);
            lp = h->ws.get("train_lp", (size_t)L * ldl * elm::dtype_size(gdt));
        }
        // the hidden layer also forms the per-row-tile partials of Z = H^T T
        const bool fuse_z = m <= elm::HIDDEN_Z_MAX_M;
        double* Zp = nullptr;
        if (fuse_z)
            Zp = (double*)h->ws.get("train_zpart",
                                    (size_t)elm::hidden_row_tiles(N) * L * m * sizeof(double));
        {
            elm::StageScope sc(&h->prof, ELM_STAGE_HIDDEN, h->stream);
            elm::launch_hidden(h->stream, ELM_F64, N, d, L, X, ldx, W, ldw, b, H64, ldh64,
                               gdt == ELM_F64 ? nullptr : lp, ldl, gdt, T, ldt, m, Zp);
        }
        if (fuse_z) {
            elm::StageScope sc(&h->prof, ELM_STAGE_RHS, h->stream);
            double* Z = (double*)h->ws.get("ps_Z", (size_t)L * m * sizeof(double));
            double* nrm = (double*)h->ws.get("ps_nrm", 2 * sizeof(double));
            elm::launch_partial_sum(h->stream, L, m, elm::hidden_row_tiles(N), Zp, Z, m, nrm, h->ws);
        }
        for (;;) {
            int64_t r = 0;
            // a factor that is not handed back lives in the handle's workspace
            elm::Workspace* pool = factor_out ? nullptr : &h->ws;
            if (gdt == ELM_F64)
                elm::check_status(h, rank_factor_impl(h, N, L, H64, ldh64, ELM_F64, ELM_SAMPLE_MAJOR,
                                                      tau_rel, &f, &r, pool));
            else
                elm::check_status(h, rank_factor_impl(h, N, L, lp, ldl, gdt, ELM_NODE_MAJOR, tau_rel,
                                                      &f, &r, pool));
            elm::check_status(h, elm_factor_get_info(f, &ti.factor));
            ti.gram_dtype = gdt;
            const bool can_escalate = gdt != ELM_F64;
            if (can_escalate && !f->reliable) {
                ti.guard = 1;
            } else {
                const elm_status ss = elm::pinv_solve_impl(h, f, m, T, ldt, H64, ldh64, ir_tol,
                                                           ir_max_iter, beta, ldbeta, &ti.solve, fuse_z,
                                                           Y, ldy, labels);
                if (ss == ELM_OK) break;
                if (ss != ELM_ERR_NO_CONVERGENCE || !can_escalate) {
                    if (info) *info = ti;
                    elm::check_status(h, ss);
                }
                ti.guard = 2;
            }
            // a guard failed: factor a higher-precision Gram of the same H
            elm::free_factor_buffers(f);
            delete f;
            f = nullptr;
            ++ti.escalations;
            gdt = elm::next_gram_dtype(gdt);
            if (gdt == ELM_F32) {
                ldl = elm::lp_ld(N);
                void* lp32 = h->ws.get("train_lp32", (size_t)L * ldl * sizeof(float));
                elm::check_status(h, elm_hidden(h, N, d, L, X, ldx, W, ldw, b, ELM_F64, nullptr, 0,
                                                lp32, ldl, ELM_F32));
                lp = lp32;
            }
        }
        if (info) *info = ti;
        if (factor_out) {
            *factor_out = f;
            f = nullptr;
        }
    });
    if (f) {
        elm::free_factor_buffers(f);
        delete f;
    }
    return st;
}

elm_status elm_train_streamed(elm_handle* h, int64_t N, int64_t d, int64_t L, int64_t m, const double* X,
                              int64_t ldx, const double* W, int64_t ldw, const double* b, const double* T,
                              int64_t ldt, elm_dtype gram_dt, int64_t chunk_rows, double tau_rel, double ir_tol,
                              int32_t ir_max_iter, double* beta, int64_t ldbeta, elm_train_info* info) {
    if (!h) return ELM_ERR_INVALID_ARG;
    elm_factor* f = nullptr;
    elm_status st = elm::guarded(h, [&] {
        REQUIRE(N >= 1 && d >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N, d and L must be >= 1");
        REQUIRE(m >= 1 && m <= 64, ELM_ERR_INVALID_ARG, "m must be in [1, 64]");
        REQUIRE(X && W && b && T && beta, ELM_ERR_INVALID_ARG, "X, W, b, T and beta must be non-null");
        REQUIRE(gram_dt == ELM_F64 || gram_dt == ELM_F32 || gram_dt == ELM_BF16 || gram_dt == ELM_F16,
                ELM_ERR_INVALID_ARG, "unknown gram dtype");
        REQUIRE(chunk_rows >= 1, ELM_ERR_INVALID_ARG, "chunk_rows must be >= 1");
        REQUIRE(N >= L, ELM_ERR_UNSUPPORTED, "the streamed form sums the column Gram over samples: N >= L");
        REQUIRE(ldx >= d && ldw >= L && ldt >= m && ldbeta >= m, ELM_ERR_SHAPE,
                "a leading dimension is smaller than its row length");
        REQUIRE(tau_rel < 1.0 && !std::isnan(tau_rel), ELM_ERR_INVALID_ARG, "tau_rel must be < 1");
        REQUIRE(ir_tol >= 0.0 && ir_tol < 1.0, ELM_ERR_INVALID_ARG, "ir_tol must be in [0, 1)");
        REQUIRE(ir_max_iter >= 0 && ir_max_iter <= 31, ELM_ERR_INVALID_ARG,
                "ir_max_iter must be in [0, 31]");
        elm::use_device(h);
        hipStream_t s = h->stream;
        elm::Workspace& ws = h->ws;
        elm::Profiler* pr = &h->prof;
        const int64_t C = std::min(chunk_rows, N);
        const int64_t nch = elm::cdiv(N, C);
        const int64_t ldl = elm::lp_ld(C);
        const bool fuse_z = m <= elm::HIDDEN_Z_MAX_M;
        // chunk buffers: the only storage of H
        double* Hc = (double*)ws.get("st_H64", (size_t)C * L * sizeof(double));
        double* M = (double*)ws.get("st_M", (size_t)L * L * sizeof(double));
        double* Mc = (double*)ws.get("st_Mc", (size_t)L * L * sizeof(double));
        double* Zparts = (double*)ws.get("st_Zparts", (size_t)nch * L * m * sizeof(double));
        double* Zp = fuse_z ? (double*)ws.get("st_Zp", (size_t)elm::hidden_row_tiles(C) * L * m * sizeof(double))
                            : nullptr;
        double* Z = (double*)ws.get("st_Z", (size_t)L * m * sizeof(double));
        double* nrm = (double*)ws.get("st_nrm", 4 * sizeof(double));
        double* E = (double*)ws.get("st_E", (size_t)C * m * sizeof(double));
        double* Gparts = (double*)ws.get("st_Gparts", (size_t)nch * L * m * sizeof(double));
        double* G = (double*)ws.get("st_G", (size_t)L * m * sizeof(double));
        double* D = (double*)ws.get("st_D", (size_t)L * m * sizeof(double));
        double* Bprev = (double*)ws.get("st_Bprev", (size_t)L * m * sizeof(double));
        auto rows_of = [&](int64_t c) { return std::min(C, N - c * C); };
        // H of chunk c: FP64 sample-major into Hc (want64) and/or the node-major
        // low-precision copy; with zc, also that chunk's H^T T partials
        auto hidden_chunk = [&](int64_t c, bool want64, void* lp, elm_dtype lpdt, bool zc) {
            const int64_t i0 = c * C, nc = rows_of(c);
            elm::StageScope sc(pr, ELM_STAGE_HIDDEN, s);
            elm::launch_hidden(s, ELM_F64, nc, d, L, X + i0 * ldx, ldx, W, ldw, b, want64 ? Hc : nullptr, L,
                               lp, ldl, lpdt, zc ? T + i0 * ldt : nullptr, ldt, zc ? m : 0, zc ? Zp : nullptr);
        };
        elm_train_info ti;
        std::memset(&ti, 0, sizeof(ti));
        elm_dtype gdt = gram_dt;
        for (;;) {
            // pass 1 over the samples: the Gram (running FP64 sum over chunks, in
            // chunk order) and H^T T (per-chunk partials summed in order)
            void* lp = nullptr;
            if (gdt != ELM_F64)
                lp = ws.get(gdt == ELM_F32 ? "st_lp32" : "st_lp16", (size_t)L * ldl * elm::dtype_size(gdt));
            int64_t kc = 0;
            for (int64_t c = 0; c < nch; ++c) {
                const int64_t i0 = c * C, nc = rows_of(c);
                const bool want64 = gdt == ELM_F64 || !fuse_z;
                hidden_chunk(c, want64, lp, gdt, fuse_z);
                {
                    elm::StageScope sc(pr, ELM_STAGE_RHS, s);
                    if (fuse_z)
                        elm::launch_partial_sum(s, L, m, elm::hidden_row_tiles(nc), Zp, Zparts + c * L * m, m, nrm,
                                                ws);
                    else
                        elm::launch_ht_times(s, nc, L, m, Hc, L, T + i0 * ldt, ldt, Zparts + c * L * m, m, nrm,
                                             ws);
                }
                double* dst = c == 0 ? M : Mc;
                if (gdt == ELM_F64)
                    elm::launch_gram_f64_cols(s, nc, L, Hc, L, dst, L, ws);
                else
                    kc = std::max(kc, elm::launch_gram_lp_nodes(s, gdt, nc, L, lp, ldl, dst, L, ws));
                if (c > 0) elm::launch_add_mat(s, L, L, Mc, L, M, L);
            }
            {
                elm::StageScope sc(pr, ELM_STAGE_RHS, s);
                elm::launch_partial_sum(s, L, m, nch, Zparts, Z, m, nrm, ws);
            }
            // the rank step and factor of the summed Gram
            f = new elm_factor();
            f->N = N;
            f->L = L;
            f->n = L;
            f->transposed = false;
            f->device = h->device;
            f->pool = &ws;
            f->gram_dtype = gdt;
            factor_gram(h, f, M, kc, tau_rel, &ws);
            (void)elm_factor_get_info(f, &ti.factor);
            ti.gram_dtype = gdt;
            const bool can_escalate = gdt != ELM_F64;
            bool converged = true;
            if (can_escalate && !f->reliable) {
                ti.guard = 1;
                converged = false;
            } else {
                // beta_0 and the refinement, each residual a second pass that
                // forms H again chunk by chunk
                std::memset(&ti.solve, 0, sizeof(ti.solve));
                ti.solve.rank = f->r;
                ti.solve.ne_residual = -1.0;
                {
                    elm::StageScope sc(pr, ELM_STAGE_SOLVE, s);
                    elm::apply_pinv(s, f, m, Z, m, nullptr, 0, beta, ldbeta, ws);
                }
                double z2 = 0;
                ELM_HIP_TRY(hipMemcpyAsync(&z2, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
                ELM_HIP_TRY(hipStreamSynchronize(s));
                if (f->pd_flag) {
                    int bad = 0;
                    ELM_HIP_TRY(hipMemcpyAsync(&bad, f->pd_flag, sizeof(int), hipMemcpyDeviceToHost, s));
                    ELM_HIP_TRY(hipStreamSynchronize(s));
                    if (bad) throw Error{ELM_ERR_NOT_PSD, "Gram of G is not positive definite"};
                }
                double res = 0, prev = 0;
                int it = 0;
                while (ir_max_iter > 0) {
                    for (int64_t c = 0; c < nch; ++c) {
                        const int64_t i0 = c * C, nc = rows_of(c);
                        hidden_chunk(c, true, nullptr, ELM_F64, false);
                        {
                            elm::StageScope sc(pr, ELM_STAGE_RESIDUAL, s);
                            elm::launch_residual(s, nc, L, m, Hc, L, T + i0 * ldt, ldt, beta, ldbeta, E, m);
                        }
                        elm::StageScope sc(pr, ELM_STAGE_RHS, s);
                        elm::launch_ht_times(s, nc, L, m, Hc, L, E, m, Gparts + c * L * m, m, nrm + 2, ws);
                    }
                    {
                        elm::StageScope sc(pr, ELM_STAGE_RHS, s);
                        elm::launch_partial_sum(s, L, m, nch, Gparts, G, m, nrm + 1, ws);
                    }
                    double g2 = 0;
                    ELM_HIP_TRY(hipMemcpyAsync(&g2, nrm + 1, sizeof(double), hipMemcpyDeviceToHost, s));
                    ELM_HIP_TRY(hipStreamSynchronize(s));
                    res = z2 > 0 ? std::sqrt(g2 / z2) : std::sqrt(g2);
                    if (it < 32) ti.solve.ne_history[it] = res;
                    if (it >= 1 && !(res < prev)) {
                        // as in elm_pinv_solve: a correction that raised the
                        // residual more than IR_RISE times is taken back
                        if (!(res <= elm::IR_RISE * prev)) {
                            ELM_HIP_TRY(hipMemcpy2DAsync(beta, (size_t)ldbeta * sizeof(double), Bprev,
                                                         (size_t)m * sizeof(double), (size_t)m * sizeof(double),
                                                         (size_t)L, hipMemcpyDeviceToDevice, s));
                            --it;
                            res = prev;
                        }
                        break;
                    }
                    if ((it >= 1 && !(res > ir_tol)) || it >= ir_max_iter) break;
                    prev = res;
                    {
                        elm::StageScope sc(pr, ELM_STAGE_SOLVE, s);
                        elm::apply_pinv(s, f, m, G, m, nullptr, 0, D, m, ws);
                    }
                    elm::launch_axpy_mat(s, L, m, D, m, beta, ldbeta, Bprev);
                    ++it;
                }
                ti.solve.iterations = it;
                ti.solve.ne_residual = ir_max_iter > 0 ? res : -1.0;
                converged = ir_max_iter == 0 || !(res > ir_tol);
                if (!converged && can_escalate) ti.guard = 2;
            }
            if (converged || !can_escalate) {
                ELM_HIP_TRY(hipStreamSynchronize(s));
                if (info) *info = ti;
                if (!converged) {
                    char msg[160];
                    std::snprintf(msg, sizeof(msg),
                                  "refinement stopped after %d iterations at relative normal-equation "
                                  "residual %.3e > ir_tol %.3e",
                                  ti.solve.iterations, ti.solve.ne_residual, ir_tol);
                    throw Error{ELM_ERR_NO_CONVERGENCE, msg};
                }
                break;
            }
            // a guard failed: the Gram again, one precision up
            elm::free_factor_buffers(f);
            delete f;
            f = nullptr;
            ++ti.escalations;
            gdt = elm::next_gram_dtype(gdt);
        }
    });
    if (f) {
        elm::free_factor_buffers(f);
        delete f;
    }
    return st;
}

elm_status elm_autotune_batch(elm_handle* h, int32_t count, const elm_problem* probs, elm_dtype gram_dt,
                              double tau_rel, double ir_tol, int32_t ir_max_iter, double* ms_before,
                              double* ms_after) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(count >= 1 && probs, ELM_ERR_INVALID_ARG, "count must be >= 1 and probs non-null");
        elm::use_device(h);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ELM_HIP_TRY(hipEventCreate(&e0));
        ELM_HIP_TRY(hipEventCreate(&e1));
        struct Ev {
            hipEvent_t a, b;
            ~Ev() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } ev{e0, e1};
        // one batch; a problem that misses ir_tol or fails its guard does not
        // stop the timing, a malformed argument does
        auto time_batch = [&]() {
            ELM_HIP_TRY(hipEventRecord(e0, h->stream));
            const elm_status st = elm_train_batched(h, count, probs, gram_dt, tau_rel, ir_tol, ir_max_iter,
                                                    nullptr, nullptr);
            if (st == ELM_ERR_INVALID_ARG || st == ELM_ERR_SHAPE || st == ELM_ERR_ALLOC || st == ELM_ERR_HIP)
                throw Error{st, h->last_error};
            ELM_HIP_TRY(hipEventRecord(e1, h->stream));
            ELM_HIP_TRY(hipEventSynchronize(e1));
            float ms = 0.f;
            ELM_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            return (double)ms;
        };
        // the batch's Gram shapes, by bucket, each with its largest problem
        struct Rep {
            int kind, dt;
            int64_t n, k;
        };
        std::vector<Rep> reps;
        for (int32_t e = 0; e < count; ++e) {
            const elm_problem& p = probs[e];
            const bool tr = p.N < p.L;
            const elm_dtype dt = tr ? ELM_F64 : gram_dt;
            const bool lp = dt == ELM_BF16 || dt == ELM_F16;
            Rep r{lp ? ELM_TUNE_GRAM_SPLITS : ELM_TUNE_GRAM_CHUNKS, (int)dt, tr ? p.N : p.L, tr ? p.L : p.N};
            bool found = false;
            for (Rep& q : reps)
                if (q.kind == r.kind && q.dt == r.dt && elm::Workspace::bucket(q.n) == elm::Workspace::bucket(r.n) &&
                    elm::Workspace::bucket(q.k) == elm::Workspace::bucket(r.k)) {
                    if (r.n * r.n * r.k > q.n * q.n * q.k) q = r;
                    found = true;
                }
            if (!found) reps.push_back(r);
        }
        const std::vector<elm_tune_entry> saved = h->ws.tune;
        auto apply = [&](int panel, double scale) {
            h->ws.tune = saved;
            h->ws.put_tune(ELM_TUNE_PANEL, -1, -1, -1, panel);
            for (const Rep& r : reps) {
                const int def = r.kind == ELM_TUNE_GRAM_SPLITS ? elm::gram_default_splits(r.k, r.n)
                                                               : elm::gram16_default_chunks(r.dt, r.n, r.k);
                const int v = std::max(1, std::min(r.kind == ELM_TUNE_GRAM_SPLITS ? 48 : 64,
                                                   (int)std::lround(def * scale)));
                h->ws.put_tune(r.kind, r.dt, r.n, r.k, v);
            }
        };
        (void)time_batch();  // untimed: buffers, tables, graphs
        const double before = time_batch();
        double best_t = before;
        int best_panel = 0;
        double best_scale = 0.0;
        for (int panel : {32, 64, 128})
            for (double scale : {0.5, 1.0, 2.0}) {
                apply(panel, scale);
                (void)time_batch();  // untimed: the candidate's tables and graphs
                const double t = time_batch();
                if (t < best_t) {
                    best_t = t;
                    best_panel = panel;
                    best_scale = scale;
                }
            }
        if (best_panel > 0 && best_t < 0.98 * before) {
            apply(best_panel, best_scale);
        } else {
            h->ws.tune = saved;
            best_t = before;
        }
        if (ms_before) *ms_before = before;
        if (ms_after) *ms_after = best_t;
    });
}

elm_status elm_probe_mfma(elm_handle* h, elm_dtype dt, int32_t shape, int32_t random_operands, double* tflops,
                          double* ms) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(dt == ELM_BF16 || dt == ELM_F64, ELM_ERR_UNSUPPORTED, "probe dtypes: BF16, FP64");
        REQUIRE(shape == 0 || (shape == 1 && dt == ELM_F64), ELM_ERR_UNSUPPORTED,
                "probe shapes: 0, and 1 (four-block 4x4x4) for FP64");
        REQUIRE(tflops, ELM_ERR_INVALID_ARG, "tflops must be non-null");
        elm::use_device(h);
        *tflops = elm::probe_mfma(h->stream, dt, shape, random_operands ? 1 : 0, ms);
    });
}

elm_status elm_probe_stream(elm_handle* h, const void* buf, int64_t bytes, double* gbs, double* ms) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(buf && gbs && bytes >= (int64_t)1 << 20, ELM_ERR_INVALID_ARG,
                "a buffer of at least 1 MiB and gbs must be given");
        REQUIRE(((uintptr_t)buf & 15) == 0, ELM_ERR_INVALID_ARG, "buf must be 16-byte aligned");
        elm::use_device(h);
        *gbs = elm::probe_stream(h->stream, buf, bytes, ms);
    });
}

elm_status elm_probe_dma(elm_handle* h, const void* buf, int64_t bytes, int32_t resident, double* gbs,
                         double* ms) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(buf && gbs, ELM_ERR_INVALID_ARG, "buf and gbs must be non-null");
        REQUIRE(bytes >= (int64_t)1024 * 4 * 32768, ELM_ERR_SHAPE, "the buffer must hold 4 stages per block");
        REQUIRE(((uintptr_t)buf & 15) == 0, ELM_ERR_INVALID_ARG, "buf must be 16-byte aligned");
        elm::use_device(h);
        *gbs = elm::probe_dma(h->stream, buf, bytes, resident ? 1 : 0, ms);
    });
}

elm_status elm_batch_get_report(const elm_handle* h, elm_batch_report* out) {
    if (!h || !out) return ELM_ERR_INVALID_ARG;
    *out = h->batch_report;
    return ELM_OK;
}

elm_status elm_train_batched(elm_handle* h, int32_t count, const elm_problem* probs,
                             elm_dtype gram_dt, double tau_rel, double ir_tol, int32_t ir_max_iter,
                             elm_train_info* infos, elm_status* statuses) {
    if (!h) return ELM_ERR_INVALID_ARG;
    std::vector<elm_status> st_all;
    std::vector<std::string> msg_all;
    elm_status st = elm::guarded(h, [&] {
        REQUIRE(count >= 0, ELM_ERR_INVALID_ARG, "count must be >= 0");
        REQUIRE(count == 0 || probs, ELM_ERR_INVALID_ARG, "probs must be non-null");
        REQUIRE(gram_dt == ELM_F64 || gram_dt == ELM_F32 || gram_dt == ELM_BF16 || gram_dt == ELM_F16,
                ELM_ERR_INVALID_ARG, "unknown gram dtype");
        REQUIRE(tau_rel < 1.0 && !std::isnan(tau_rel), ELM_ERR_INVALID_ARG, "tau_rel must be < 1");
        REQUIRE(ir_tol >= 0.0 && ir_tol < 1.0, ELM_ERR_INVALID_ARG, "ir_tol must be in [0, 1)");
        REQUIRE(ir_max_iter >= 0 && ir_max_iter <= 31, ELM_ERR_INVALID_ARG,
                "ir_max_iter must be in [0, 31]");
        for (int32_t e = 0; e < count; ++e) {
            const elm_problem& p = probs[e];
            const std::string at = "problem " + std::to_string(e) + ": ";
            REQUIRE(p.N >= 1 && p.d >= 1 && p.L >= 1 && p.m >= 1 && p.m <= 64, ELM_ERR_INVALID_ARG,
                    at + "N, d, L must be >= 1 and m in [1, 64]");
            REQUIRE(p.X && p.W && p.b && p.T && p.H64 && p.beta, ELM_ERR_INVALID_ARG,
                    at + "a pointer is null");
            REQUIRE(p.ldx >= p.d && p.ldw >= p.L && p.ldt >= p.m && p.ldh64 >= p.L && p.ldbeta >= p.m,
                    ELM_ERR_SHAPE, at + "a leading dimension is smaller than its row length");
        }
        h->batch_report = elm_batch_report{};
        if (count == 0) return;
        elm::use_device(h);
        struct ReportFill {
            elm_handle* h;
            int64_t c0, l0, s0;
            ~ReportFill() {
                h->batch_report.graph_captures = (int32_t)(h->ws.graph_captures - c0);
                h->batch_report.graph_launches = (int32_t)(h->ws.graph_launches - l0);
                h->batch_report.batch_stream_syncs = (int32_t)(h->ws.host_syncs - s0);
            }
        } report_fill{h, h->ws.graph_captures, h->ws.graph_launches, h->ws.host_syncs};
        const int nw = count < h->batch_workers ? count : h->batch_workers;
        while ((int)h->workers.size() < nw) {
            hipStream_t ws_stream = nullptr;
            ELM_HIP_TRY(hipStreamCreateWithFlags(&ws_stream, hipStreamNonBlocking));
            elm_handle* w = nullptr;
            if (elm_create(&w, ws_stream) != ELM_OK) {
                (void)hipStreamDestroy(ws_stream);
                throw elm::Error{ELM_ERR_HIP, "cannot create a worker handle"};
            }
            w->owns_stream = true;
            h->workers.push_back(w);
        }
        for (int w = 0; w < nw; ++w) {
            // the workers take the handle's options and tuned schedules, so a
            // problem gives the same bits wherever it runs
            h->workers[w]->full_rank_min_order = h->full_rank_min_order;
            h->workers[w]->ws.tune = h->ws.tune;
        }
        // the workers start after the work already queued on the caller's stream
        hipEvent_t ev = nullptr;
        ELM_HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        ELM_HIP_TRY(hipEventRecord(ev, h->stream));
        for (int w = 0; w < nw; ++w) ELM_HIP_TRY(hipStreamWaitEvent(h->workers[w]->stream, ev, 0));
        if (!h->batch_stream)  // default priority, non-blocking
            ELM_HIP_TRY(hipStreamCreateWithFlags(&h->batch_stream, hipStreamNonBlocking));
        ELM_HIP_TRY(hipStreamWaitEvent(h->batch_stream, ev, 0));
        // the shared launches of the batch (phases 1 to 3) run on this stream
        hipStream_t ps = h->batch_stream;
        // workers take problems longest-first by the Gram's cost N n min(N, L)
        auto cost = [&](int32_t e) {
            const double n = (double)std::min(probs[e].N, probs[e].L);
            return (double)std::max(probs[e].N, probs[e].L) * n * n + 2.0e5 * n;
        };
        st_all.assign(count, ELM_OK);
        msg_all.assign(count, std::string());
        std::vector<elm_train_info> info_all(count);
        for (auto& ti : info_all) std::memset(&ti, 0, sizeof(ti));
        // stage timers of the workers follow the handle's (summed into it below)
        for (int w = 0; w < nw; ++w) h->workers[w]->prof.on = h->prof.on;

        // Per problem: the Gram's order and precision, and where the first
        // phase leaves the Gram, Z = H^T T, ||Z||^2 and the largest diagonal.
        struct Item {
            elm_dtype gdt;
            int64_t n, kc;
            bool transposed, fuse_z, ok;
            double *M, *Z, *nrm;
        };
        std::vector<Item> items(count);
        auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
        // Problems run in groups whose Grams and factorisation scratch
        // (about 4 n^2 doubles each) fit in BATCH_GROUP_BYTES.
        std::vector<std::vector<int32_t>> groups(1);
        size_t gbytes = 0;
        for (int32_t e = 0; e < count; ++e) {
            const elm_problem& p = probs[e];
            Item& it = items[e];
            it.transposed = p.N < p.L;
            it.n = it.transposed ? p.N : p.L;
            it.gdt = it.transposed ? ELM_F64 : gram_dt;
            it.fuse_z = p.m <= elm::HIDDEN_Z_MAX_M;
            it.kc = 0;
            it.ok = true;
            size_t need = 4 * al((size_t)it.n * it.n * sizeof(double)) +
                          (size_t)256 * it.n * sizeof(double);
            if (!it.transposed && it.fuse_z)  // the shared phase-1 buffers
                need += al((size_t)p.L * elm::lp_ld(p.N) * elm::dtype_size(it.gdt)) +
                        al((size_t)elm::hidden_row_tiles(p.N) * p.L * p.m * sizeof(double)) +
                        al((size_t)p.L * p.L * sizeof(double));
            if (!groups.back().empty() && gbytes + need > elm::BATCH_GROUP_BYTES) {
                groups.emplace_back();
                gbytes = 0;
            }
            groups.back().push_back(e);
            gbytes += need;
        }
        hipEvent_t ev2 = nullptr;
        ELM_HIP_TRY(hipEventCreateWithFlags(&ev2, hipEventDisableTiming));
        struct EvGuard {
            hipEvent_t e;
            ~EvGuard() { (void)hipEventDestroy(e); }
        } ev2_guard{ev2};
        // runs body(worker handle, problem) for every problem of the group on
        // the workers (longest first), recording failures per problem
        auto run_workers = [&](const std::vector<int32_t>& grp, auto&& body) {
            std::vector<std::vector<int32_t>> lists(nw);
            std::vector<double> load(nw, 0.0);
            std::vector<int32_t> ord(grp);
            std::stable_sort(ord.begin(), ord.end(),
                             [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
            for (int32_t e : ord) {
                if (!items[e].ok) continue;
                const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                lists[w].push_back(e);
                load[w] += cost(e);
            }
            std::vector<std::thread> threads;
            for (int w = 0; w < nw; ++w) {
                threads.emplace_back([&, w] {
                    elm_handle* wh = h->workers[w];
                    for (int32_t e : lists[w]) {
                        try {
                            body(wh, e);
                        } catch (const elm::Error& err) {
                            st_all[e] = err.st;
                            msg_all[e] = err.msg;
                            items[e].ok = false;
                        } catch (const std::bad_alloc&) {
                            st_all[e] = ELM_ERR_ALLOC;
                            msg_all[e] = "host allocation failed";
                            items[e].ok = false;
                        } catch (const std::exception& x) {
                            st_all[e] = ELM_ERR_HIP;
                            msg_all[e] = x.what();
                            items[e].ok = false;
                        }
                    }
                });
            }
            for (auto& t : threads) t.join();
        };
        // stream order: each worker waits for `from`, or `from` for every worker
        auto workers_wait = [&](hipStream_t from) {
            ELM_HIP_TRY(hipEventRecord(ev2, from));
            for (int w = 0; w < nw; ++w) ELM_HIP_TRY(hipStreamWaitEvent(h->workers[w]->stream, ev2, 0));
        };
        auto wait_workers = [&](hipStream_t into) {
            for (int w = 0; w < nw; ++w) {
                ELM_HIP_TRY(hipEventRecord(ev2, h->workers[w]->stream));
                ELM_HIP_TRY(hipStreamWaitEvent(into, ev2, 0));
            }
        };

        // Phase 1 of problems g1 in shared launches on stream s: the hidden
        // layers (H, the low-precision copy, the row-tile partials of
        // Z = H^T T), Z and ||Z||^2, the Grams and their largest diagonal
        // entries; the kernels, tiles and splits of the single-problem launches.
        // The programs' host blobs must live until their uploads are done (the
        // caller keeps them to its next synchronisation).
        auto run_phase1_grouped = [&](elm_handle* hh, hipStream_t s, const std::vector<int32_t>& g1,
                                      const std::vector<int32_t>& slot, double* dmaxs,
                                      std::vector<elm::GroupProgram>& progs) {
            const size_t P = g1.size();
            std::vector<elm::HiddenDesc> hd(P);
            std::vector<elm::PsumDesc> sd(P);
            std::vector<elm::GramDesc> gd(P);
            std::vector<size_t> o_lp(P), o_zp(P), o_p2(P), o_sq(P), o_gp(P);
            std::vector<int64_t> kc(P, 0);
            size_t off = 0;
            for (size_t j = 0; j < P; ++j) {
                const elm_problem& p = probs[g1[j]];
                const Item& it = items[g1[j]];
                const int64_t nrt = elm::hidden_row_tiles(p.N);
                o_lp[j] = off;
                if (it.gdt != ELM_F64) off += al((size_t)p.L * elm::lp_ld(p.N) * elm::dtype_size(it.gdt));
                o_zp[j] = off;
                off += al((size_t)nrt * p.L * p.m * sizeof(double));
                o_p2[j] = off;
                off += al(std::max<size_t>(elm::psum_part2_doubles(p.L, p.m, nrt), 1) * sizeof(double));
                o_sq[j] = off;
                off += al(elm::refine_sq_doubles(p.L, p.m) * sizeof(double));
                o_gp[j] = off;
                off += al(elm::gram_group_plan(s, it.gdt, p.N, p.L, gd[j], hh->ws, &kc[j]));
            }
            char* arena = (char*)hh->ws.get("bt_phase1", off);
            for (size_t j = 0; j < P; ++j) {
                const int32_t e = g1[j];
                const elm_problem& p = probs[e];
                Item& it = items[e];
                void* lp = it.gdt != ELM_F64 ? (void*)(arena + o_lp[j]) : nullptr;
                double* Zp = (double*)(arena + o_zp[j]);
                elm::HiddenDesc& h1 = hd[j];
                h1.N = p.N;
                h1.d = p.d;
                h1.L = p.L;
                h1.X = (const double*)p.X;
                h1.ldx = p.ldx;
                h1.W = (const double*)p.W;
                h1.ldw = p.ldw;
                h1.b = (const double*)p.b;
                h1.H = p.H64;
                h1.ldh = p.ldh64;
                h1.Hlp = lp;
                h1.ldlp = elm::lp_ld(p.N);
                h1.lp_dt = it.gdt;
                h1.T = p.T;
                h1.ldt = p.ldt;
                h1.m = (int)p.m;
                h1.Zp = Zp;
                elm::PsumDesc& s1 = sd[j];
                s1.L = p.L;
                s1.m = p.m;
                s1.nchunk = elm::hidden_row_tiles(p.N);
                s1.part = Zp;
                s1.part2 = (double*)(arena + o_p2[j]);
                s1.G = it.Z;
                s1.sq = (double*)(arena + o_sq[j]);
                s1.nrm2 = it.nrm;
                elm::GramDesc& g = gd[j];
                g.A = it.gdt == ELM_F64 ? (const void*)p.H64 : (const void*)lp;
                g.ld = it.gdt == ELM_F64 ? p.ldh64 : elm::lp_ld(p.N);
                g.part = arena + o_gp[j];
                g.M = it.M;
                g.ldm = it.n;
                g.dmax = dmaxs + slot[e];
                it.kc = it.gdt != ELM_F64 ? kc[j] : 0;
            }
            progs.assign(3, elm::GroupProgram());
            std::vector<int64_t> nb(P);
            for (size_t j = 0; j < P; ++j) nb[j] = elm::hidden_group_blocks(hd[j]);
            progs[0].add(hd, nb, [](hipStream_t st, const void* d, const elm::GroupSched& g) {
                elm::launch_hidden_grouped(st, (const elm::HiddenDesc*)d, g);
            });
            for (int stage = 0; stage < 3; ++stage) {
                for (size_t j = 0; j < P; ++j) nb[j] = elm::partial_sum_group_blocks(stage, sd[j]);
                progs[1].add(sd, nb, [stage](hipStream_t st, const void* d, const elm::GroupSched& g) {
                    elm::launch_partial_sum_grouped(st, stage, (const elm::PsumDesc*)d, g);
                });
            }
            const int kind = gd[0].kind;  // one Gram type per batch
            for (int stage = 0; stage < 3; ++stage) {
                for (size_t j = 0; j < P; ++j) nb[j] = elm::gram_group_blocks(stage, gd[j]);
                progs[2].add(gd, nb, [stage, kind](hipStream_t st, const void* d, const elm::GroupSched& g) {
                    elm::launch_gram_grouped(st, stage, kind, (const elm::GramDesc*)d, g);
                });
            }
            const char* names[3] = {"bt_p1_hidden", "bt_p1_rhs", "bt_p1_gram"};
            const int stages[3] = {ELM_STAGE_HIDDEN, ELM_STAGE_RHS, ELM_STAGE_GRAM};
            for (int k = 0; k < 3; ++k) {
                elm::StageScope sc(&hh->prof, stages[k], s);
                progs[k].run(s, hh->ws, names[k]);
            }
        };

        h->batch_report.groups = (int32_t)groups.size();
        for (const std::vector<int32_t>& grp : groups) {
            // phase 1: H, Z = H^T T and the Gram of every problem
            size_t mb = 0, zb = 0;
            for (int32_t e : grp) {
                mb += al((size_t)items[e].n * items[e].n * sizeof(double));
                zb += al((size_t)probs[e].L * probs[e].m * sizeof(double));
            }
            char* Marena = (char*)h->ws.get("bt_M", mb);
            char* Zarena = (char*)h->ws.get("bt_Z", zb);
            double* nrms = (double*)h->ws.get("bt_nrm", grp.size() * 2 * sizeof(double));
            double* dmaxs = (double*)h->ws.get("bt_dmax", grp.size() * sizeof(double));
            {
                size_t mo = 0, zo = 0;
                for (size_t i = 0; i < grp.size(); ++i) {
                    Item& it = items[grp[i]];
                    it.M = (double*)(Marena + mo);
                    it.Z = (double*)(Zarena + zo);
                    it.nrm = nrms + 2 * i;
                    mo += al((size_t)it.n * it.n * sizeof(double));
                    zo += al((size_t)probs[grp[i]].L * probs[grp[i]].m * sizeof(double));
                }
            }
            std::vector<int32_t> slot(count, -1);
            for (size_t i = 0; i < grp.size(); ++i) slot[grp[i]] = (int32_t)i;
            // phase 1, shared launches (batch stream): the problems with
            // N >= L and H^T T from the hidden layer
            std::vector<elm::GroupProgram> p1progs;  // until the synchronisation of phase 2
            {
                std::vector<int32_t> g1;
                for (int32_t e : grp)
                    if (items[e].ok && !items[e].transposed && items[e].fuse_z) g1.push_back(e);
                if (!g1.empty()) {
                    try {
                        run_phase1_grouped(h, ps, g1, slot, dmaxs, p1progs);
                    } catch (const elm::Error& err) {
                        for (int32_t e : g1) {
                            st_all[e] = err.st;
                            msg_all[e] = err.msg;
                            items[e].ok = false;
                        }
                    }
                }
            }
            // phase 1 (workers): the others
            run_workers(grp, [&](elm_handle* wh, int32_t e) {
                const elm_problem& p = probs[e];
                Item& it = items[e];
                if (!it.transposed && it.fuse_z) return;  // shared launches
                hipStream_t ws = wh->stream;
                void* lp = nullptr;
                if (it.gdt != ELM_F64)
                    lp = wh->ws.get("train_lp", (size_t)p.L * elm::lp_ld(p.N) * elm::dtype_size(it.gdt));
                double* Zp = nullptr;
                if (it.fuse_z)
                    Zp = (double*)wh->ws.get("train_zpart", (size_t)elm::hidden_row_tiles(p.N) * p.L *
                                                                p.m * sizeof(double));
                {
                    elm::StageScope sc(&wh->prof, ELM_STAGE_HIDDEN, ws);
                    elm::launch_hidden(ws, ELM_F64, p.N, p.d, p.L, p.X, p.ldx, p.W, p.ldw, p.b, p.H64,
                                       p.ldh64, lp, elm::lp_ld(p.N), it.gdt, p.T, p.ldt, p.m, Zp);
                }
                if (it.fuse_z) {
                    elm::StageScope sc(&wh->prof, ELM_STAGE_RHS, ws);
                    elm::launch_partial_sum(ws, p.L, p.m, elm::hidden_row_tiles(p.N), Zp, it.Z, p.m,
                                            it.nrm, wh->ws);
                }
                if (it.gdt == ELM_F64) {
                    if (it.transposed)
                        elm::launch_gram_f64_rows(ws, p.N, p.L, p.H64, p.ldh64, it.M, it.n, wh->ws);
                    else
                        elm::launch_gram_f64_cols(ws, p.N, p.L, p.H64, p.ldh64, it.M, it.n, wh->ws);
                } else {
                    it.kc = elm::launch_gram_lp_nodes(ws, it.gdt, p.N, p.L, lp, elm::lp_ld(p.N), it.M, it.n,
                                                      wh->ws);
                }
                elm::launch_diag_max(ws, it.n, it.M, it.n, dmaxs + slot[e]);
            });
            // phase 2 runs on the batch stream (a created stream, so its fixed
            // launch sequences can be replayed as HIP graphs)
            wait_workers(ps);

            // phase 2: all rank decisions in shared launches
            std::vector<double> hdmax(grp.size());
            ELM_HIP_TRY(hipMemcpyAsync(hdmax.data(), dmaxs, grp.size() * sizeof(double),
                                       hipMemcpyDeviceToHost, ps));
            ELM_HIP_TRY(hipStreamSynchronize(ps));
            ++h->ws.host_syncs;
            std::vector<elm::PcholProblem> pc;
            std::vector<int32_t> pc_of(count, -1);
            for (size_t i = 0; i < grp.size(); ++i) {
                const int32_t e = grp[i];
                Item& it = items[e];
                if (!it.ok) continue;
                if (!std::isfinite(hdmax[i])) {
                    st_all[e] = ELM_ERR_NOT_PSD;
                    msg_all[e] = "Gram has a non-finite diagonal entry";
                    it.ok = false;
                    continue;
                }
                // the threshold of elm_rank_factor
                const int64_t K = it.transposed ? probs[e].L : probs[e].N;
                elm::PcholProblem q;
                q.n = it.n;
                q.M = it.M;
                q.ldm = it.n;
                q.tau = (tau_rel > 0 ? tau_rel : 16.0 * (double)(it.n + K) * std::ldexp(1.0, -53)) *
                        hdmax[i];
                pc_of[e] = (int32_t)pc.size();
                pc.push_back(q);
            }
            {
                elm::StageScope sc(&h->prof, ELM_STAGE_RANK, ps);
                elm::pivoted_cholesky_grouped(ps, pc, h->ws);   // reads the ranks back
            }
            workers_wait(ps);

            // Rank decisions: the rule of elm_rank_factor's diagnostics
            auto reliable_of = [&](int32_t e) {
                const Item& it = items[e];
                const elm::PcholProblem& q = pc[pc_of[e]];
                const double hd = hdmax[slot[e]];
                const double nf = elm::schur_noise_floor(it.gdt, it.n, std::max(probs[e].N, probs[e].L),
                                                         it.kc) * hd;
                return (q.rank == 0 || q.stats[0] >= 2.0 * nf) &&
                       (q.rank == it.n || q.stats[1] >= -2.0 * nf);
            };
            // Problems whose solve and refinement run grouped (phase 3b):
            // non-transposed, H^T T from the hidden layer, rank >= 1, a rank
            // decision that stands.  Their factors live in one arena.
            auto factor_bytes = [&](int64_t r, int64_t n) {
                const int64_t c = n - r, q = std::min(r, c);
                size_t b = al((size_t)r * n * sizeof(double)) + 2 * al((size_t)r * r * sizeof(double));
                if (c > 0) b += 2 * al((size_t)r * c * sizeof(double));
                if (q > 0) b += 2 * al((size_t)q * q * sizeof(double));
                return b;
            };
            std::vector<size_t> foff(count, 0), fsize(count, 0);
            std::vector<char> grouped(count, 0);
            size_t fbytes = 0;
            for (int32_t e : grp) {
                const Item& it = items[e];
                if (!it.ok || pc_of[e] < 0) continue;
                const elm::PcholProblem& q = pc[pc_of[e]];
                if (q.bad || it.transposed || !it.fuse_z || q.rank == 0) continue;
                if (it.gdt != ELM_F64 && !reliable_of(e)) continue;  // escalates at once
                grouped[e] = 1;
                foff[e] = fbytes;
                fsize[e] = factor_bytes(q.rank, it.n);
                fbytes += fsize[e];
            }
            char* farena = fbytes ? (char*)h->ws.get("bt_factors", fbytes) : nullptr;
            std::vector<std::unique_ptr<elm_factor>> gfac(count);

            for (int32_t e : grp) {
                if (grouped[e]) ++h->batch_report.grouped_problems;
                else if (items[e].ok) ++h->batch_report.worker_problems;
            }
            // a guard failed: train problem e again from a higher-precision Gram
            auto escalate = [&](elm_handle* wh, int32_t e, int guard) {
                const elm_problem& p = probs[e];
                elm_train_info t2;
                std::memset(&t2, 0, sizeof(t2));
                const elm_status s2 =
                    elm_train(wh, p.N, p.d, p.L, p.m, p.X, p.ldx, p.W, p.ldw, p.b, p.T, p.ldt,
                              elm::next_gram_dtype(items[e].gdt), p.H64, p.ldh64, nullptr, 0, tau_rel,
                              ir_tol, ir_max_iter, p.beta, p.ldbeta, nullptr, 0, nullptr, &t2, nullptr);
                t2.escalations += 1;
                if (!t2.guard) t2.guard = guard;
                info_all[e] = t2;
                elm::check_status(wh, s2);
            };

            // phase 3a (workers): the problems that do not run grouped
            run_workers(grp, [&](elm_handle* wh, int32_t e) {
                if (grouped[e]) return;
                const elm_problem& p = probs[e];
                Item& it = items[e];
                const elm::PcholProblem& q = pc[pc_of[e]];
                hipStream_t ws = wh->stream;
                elm_train_info& ti = info_all[e];
                if (q.bad) throw elm::Error{ELM_ERR_NOT_PSD, "Gram has a non-finite diagonal entry"};
                std::unique_ptr<elm_factor> fp(new elm_factor());
                elm_factor* f = fp.get();
                struct BufGuard {
                    elm_factor* f;
                    ~BufGuard() { elm::free_factor_buffers(f); }
                } bg{f};
                f->N = p.N;
                f->L = p.L;
                f->n = it.n;
                f->transposed = it.transposed;
                f->device = h->device;
                f->gram_dtype = it.gdt;
                f->tau = q.tau;
                f->r = q.rank;
                f->pool = &wh->ws;
                f->piv = (int32_t*)elm::factor_alloc(f, "piv", (size_t)it.n * sizeof(int32_t));
                ELM_HIP_TRY(hipMemcpyAsync(f->piv, q.piv, (size_t)it.n * sizeof(int32_t),
                                           hipMemcpyDeviceToDevice, ws));
                if (f->r > 0) {
                    f->R = (double*)elm::factor_alloc(f, "R", (size_t)f->r * it.n * sizeof(double));
                    elm::launch_gather_rows(ws, f->r, it.n, q.Rorig, it.n, q.piv, f->R, it.n);
                }
                const double hd = hdmax[slot[e]];
                f->last_pivot = q.stats[0];
                f->first_rejected = q.stats[1];
                f->max_diag = hd;
                f->noise_floor =
                    elm::schur_noise_floor(it.gdt, it.n, p.N > p.L ? p.N : p.L, it.kc) * hd;
                f->reliable = reliable_of(e);
                elm::check_status(wh, elm_factor_get_info(f, &ti.factor));
                ti.gram_dtype = it.gdt;
                const bool can_escalate = it.gdt != ELM_F64;
                if (can_escalate && !f->reliable) {
                    escalate(wh, e, 1);
                    return;
                }
                {
                    elm::StageScope sc(&wh->prof, ELM_STAGE_FACTOR, ws);
                    elm::build_factor_tail(ws, f, wh->ws, /*wait=*/false);
                }
                if (it.fuse_z) {
                    double* Z = (double*)wh->ws.get("ps_Z", (size_t)p.L * p.m * sizeof(double));
                    double* nrm = (double*)wh->ws.get("ps_nrm", 2 * sizeof(double));
                    ELM_HIP_TRY(hipMemcpyAsync(Z, it.Z, (size_t)p.L * p.m * sizeof(double),
                                               hipMemcpyDeviceToDevice, ws));
                    ELM_HIP_TRY(hipMemcpyAsync(nrm, it.nrm, sizeof(double), hipMemcpyDeviceToDevice, ws));
                }
                const elm_status ss =
                    elm::pinv_solve_impl(wh, f, p.m, p.T, p.ldt, p.H64, p.ldh64, ir_tol, ir_max_iter,
                                         p.beta, p.ldbeta, &ti.solve, it.fuse_z);
                if (ss == ELM_OK) return;
                if (ss != ELM_ERR_NO_CONVERGENCE || !can_escalate) elm::check_status(wh, ss);
                escalate(wh, e, 2);
            });

            // phase 3b (one stream): factor tails, beta and refinement of the
            // grouped problems
            wait_workers(ps);
            {
                std::vector<elm_factor*> tf;
                std::vector<const double*> rorig;
                std::vector<int32_t> tf_of;
                for (int32_t e : grp) {
                    if (!grouped[e]) continue;
                    const elm_problem& p = probs[e];
                    const Item& it = items[e];
                    const elm::PcholProblem& q = pc[pc_of[e]];
                    std::unique_ptr<elm_factor> f(new elm_factor());
                    f->N = p.N;
                    f->L = p.L;
                    f->n = it.n;
                    f->transposed = false;
                    f->device = h->device;
                    f->gram_dtype = it.gdt;
                    f->tau = q.tau;
                    f->r = q.rank;
                    // the grouped factorisation's pivots stay valid until the next group
                    f->arena = farena + foff[e];
                    f->arena_left = fsize[e];
                    f->piv = const_cast<int32_t*>(q.piv);
                    f->R = (double*)elm::factor_alloc(f.get(), "R", (size_t)f->r * it.n * sizeof(double));
                    const double hd = hdmax[slot[e]];
                    f->last_pivot = q.stats[0];
                    f->first_rejected = q.stats[1];
                    f->max_diag = hd;
                    f->noise_floor =
                        elm::schur_noise_floor(it.gdt, it.n, std::max(p.N, p.L), it.kc) * hd;
                    f->reliable = reliable_of(e);
                    elm_train_info& ti = info_all[e];
                    elm::check_status(h, elm_factor_get_info(f.get(), &ti.factor));
                    ti.gram_dtype = it.gdt;
                    tf.push_back(f.get());
                    rorig.push_back(q.Rorig);
                    tf_of.push_back(e);
                    gfac[e] = std::move(f);
                }
                try {
                    std::vector<int> bad;
                    {
                        elm::StageScope sc(&h->prof, ELM_STAGE_FACTOR, ps);
                        bad = elm::build_factor_tails_grouped(ps, tf, rorig, h->ws);   // reads the flags back
                    }
                    for (size_t j = 0; j < tf_of.size(); ++j)
                        if (bad[j]) {
                            const int32_t e = tf_of[j];
                            st_all[e] = ELM_ERR_NOT_PSD;
                            msg_all[e] = "Gram of G is not positive definite";
                            items[e].ok = false;
                        }
                } catch (const elm::Error& err) {
                    for (int32_t e : tf_of) {
                        st_all[e] = err.st;
                        msg_all[e] = err.msg;
                        items[e].ok = false;
                    }
                }
            }
            std::vector<elm::GroupedSolve> gs;
            std::vector<int32_t> gs_of;
            for (int32_t e : grp) {
                if (!gfac[e] || !items[e].ok) continue;
                const elm_problem& p = probs[e];
                elm::GroupedSolve g;
                g.f = gfac[e].get();
                g.m = p.m;
                g.H64 = p.H64;
                g.ldh64 = p.ldh64;
                g.T = p.T;
                g.ldt = p.ldt;
                g.beta = p.beta;
                g.ldbeta = p.ldbeta;
                g.Z = items[e].Z;
                g.z2 = items[e].nrm;   // ||Z||^2 from phase 1, on the device
                g.info = &info_all[e].solve;
                gs.push_back(g);
                gs_of.push_back(e);
            }
            std::vector<int32_t> esc;
            try {
                elm::refine_grouped(h, ps, gs, ir_tol, ir_max_iter);
                for (size_t j = 0; j < gs.size(); ++j) {
                    const int32_t e = gs_of[j];
                    if (gs[j].status == ELM_OK) continue;
                    if (items[e].gdt != ELM_F64) {
                        esc.push_back(e);
                    } else {
                        st_all[e] = gs[j].status;
                        msg_all[e] = gs[j].msg;
                        items[e].ok = false;
                    }
                }
            } catch (const elm::Error& err) {
                for (int32_t e : gs_of) {
                    st_all[e] = err.st;
                    msg_all[e] = err.msg;
                    items[e].ok = false;
                }
            }
            for (auto& f : gfac)
                if (f) elm::free_factor_buffers(f.get());
            // phase 3c (workers): problems whose grouped refinement missed ir_tol
            if (!esc.empty()) {
                workers_wait(ps);
                run_workers(esc, [&](elm_handle* wh, int32_t e) { escalate(wh, e, 2); });
            }
        }
        if (h->prof.on) {
            for (int w = 0; w < nw; ++w) {
                elm::Profiler& wp = h->workers[w]->prof;
                wp.resolve();
                for (int i = 0; i < ELM_STAGE_COUNT; ++i) {
                    h->prof.ms[i] += wp.ms[i];
                    h->prof.cnt[i] += wp.cnt[i];
                    wp.ms[i] = 0;
                    wp.cnt[i] = 0;
                }
            }
        }
        // the caller's stream continues after the workers
        for (int w = 0; w < nw; ++w) {
            ELM_HIP_TRY(hipEventRecord(ev, h->workers[w]->stream));
            ELM_HIP_TRY(hipStreamWaitEvent(h->stream, ev, 0));
        }
        ELM_HIP_TRY(hipEventDestroy(ev));
        for (int32_t e = 0; e < count; ++e)
            if (info_all[e].escalations > 0) ++h->batch_report.escalations;
        if (infos) std::memcpy(infos, info_all.data(), (size_t)count * sizeof(elm_train_info));
        if (statuses) std::memcpy(statuses, st_all.data(), (size_t)count * sizeof(elm_status));
        for (int32_t e = 0; e < count; ++e)
            if (st_all[e] != ELM_OK)
                throw elm::Error{st_all[e], "problem " + std::to_string(e) + ": " + msg_all[e]};
    });
    return st;
}

}  // extern "C"

extern "C" {

elm_status elm_predict(elm_handle* h, int64_t N, int64_t d, int64_t L, int64_t m, const void* X,
                       int64_t ldx, const void* W, int64_t ldw, const void* b, elm_dtype dt,
                       const double* beta, int64_t ldbeta, void* Y, int64_t ldy, int32_t* labels) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(N >= 1 && d >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N, d and L must be >= 1");
        REQUIRE(m >= 1 && m <= 64, ELM_ERR_INVALID_ARG, "m must be in [1, 64]");
        REQUIRE(X && W && b && beta, ELM_ERR_INVALID_ARG, "X, W, b and beta must be non-null");
        REQUIRE(Y || labels, ELM_ERR_INVALID_ARG, "at least one of Y and labels must be non-null");
        REQUIRE(dt == ELM_F64 || dt == ELM_F32, ELM_ERR_UNSUPPORTED, "dt must be ELM_F64 or ELM_F32");
        REQUIRE(ldx >= d && ldw >= L && ldbeta >= m, ELM_ERR_SHAPE, "leading dimension too small");
        if (Y) REQUIRE(ldy >= m, ELM_ERR_SHAPE, "ldy < m");
        elm::use_device(h);
        elm::StageScope sc(&h->prof, ELM_STAGE_PREDICT, h->stream);
        elm::launch_predict(h->stream, dt, N, d, L, m, X, ldx, W, ldw, b, beta, ldbeta, Y, ldy,
                            labels, h->ws);
    });
}

elm_status elm_predict_hidden(elm_handle* h, int64_t N, int64_t L, int64_t m, const double* H,
                              int64_t ldh, const double* beta, int64_t ldbeta, double* Y, int64_t ldy,
                              int32_t* labels) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(N >= 1 && L >= 1, ELM_ERR_INVALID_ARG, "N and L must be >= 1");
        REQUIRE(m >= 1 && m <= 64, ELM_ERR_INVALID_ARG, "m must be in [1, 64]");
        REQUIRE(H && beta, ELM_ERR_INVALID_ARG, "H and beta must be non-null");
        REQUIRE(Y || labels, ELM_ERR_INVALID_ARG, "at least one of Y and labels must be non-null");
        REQUIRE(ldh >= L && ldbeta >= m, ELM_ERR_SHAPE, "leading dimension too small");
        if (Y) REQUIRE(ldy >= m, ELM_ERR_SHAPE, "ldy < m");
        elm::use_device(h);
        elm::StageScope sc(&h->prof, ELM_STAGE_PREDICT, h->stream);
        elm::launch_hidden_output(h->stream, N, L, m, H, ldh, beta, ldbeta, Y, ldy, labels);
    });
}

elm_status elm_set_option(elm_handle* h, elm_option opt, int64_t value) {
    if (!h) return ELM_ERR_INVALID_ARG;
    switch (opt) {
        case ELM_OPT_FULL_RANK_MIN_ORDER:
            h->full_rank_min_order = value;
            return ELM_OK;
        case ELM_OPT_BATCH_WORKERS:
            if (value < 1 || value > 16) {
                h->last_error = "batch workers must be in [1, 16]";
                return ELM_ERR_INVALID_ARG;
            }
            h->batch_workers = (int)value;
            return ELM_OK;
    }
    h->last_error = "unknown option";
    return ELM_ERR_INVALID_ARG;
}

elm_status elm_get_option(const elm_handle* h, elm_option opt, int64_t* value) {
    if (!h || !value) return ELM_ERR_INVALID_ARG;
    switch (opt) {
        case ELM_OPT_FULL_RANK_MIN_ORDER:
            *value = h->full_rank_min_order;
            return ELM_OK;
        case ELM_OPT_BATCH_WORKERS:
            *value = h->batch_workers;
            return ELM_OK;
    }
    return ELM_ERR_INVALID_ARG;
}

elm_status elm_profile_enable(elm_handle* h, int enable) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        elm::use_device(h);
        if (enable) {
            h->prof.resolve();
            for (int i = 0; i < ELM_STAGE_COUNT; ++i) {
                h->prof.ms[i] = 0;
                h->prof.cnt[i] = 0;
            }
        }
        h->prof.on = enable != 0;
    });
}

elm_status elm_profile_read(elm_handle* h, elm_stage_times* out) {
    if (!h) return ELM_ERR_INVALID_ARG;
    return elm::guarded(h, [&] {
        REQUIRE(out, ELM_ERR_INVALID_ARG, "out must be non-null");
        elm::use_device(h);
        h->prof.resolve();
        for (int i = 0; i < ELM_STAGE_COUNT; ++i) {
            out->ms[i] = h->prof.ms[i];
            out->count[i] = h->prof.cnt[i];
        }
    });
}

}  // extern "C"
