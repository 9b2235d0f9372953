// Internal declarations shared by the libelm translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>
#include <functional>
#include <cstring>

#include "../../include/elm.h"

namespace elm {

// ---------------------------------------------------------------------------
// vector types used by the MFMA builtins
// ---------------------------------------------------------------------------
typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// 16 x 16 x 4 MFMA with one element per lane for A (16 x 4) and B (4 x 16):
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].  The 16 x 16 result
// sits in 4 registers per lane; row(l, v) is the row of register v of lane l,
// the column is l % 16.  The FP64 and FP32 instructions place rows
// differently (measured on gfx950).
// ---------------------------------------------------------------------------
template <typename T> struct Mfma16;
template <> struct Mfma16<double> {
    typedef d4v acc_t;
    static __device__ inline acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int v) { return 4 * v + (lane >> 4); }
};
template <> struct Mfma16<float> {
    typedef f4v acc_t;
    static __device__ inline acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ inline int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
struct Error {
    elm_status st;
    std::string msg;
};

#define ELM_HIP_TRY(expr)                                                             \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::elm::Error{ELM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define ELM_LAUNCH_CHECK() ELM_HIP_TRY(hipGetLastError())

// ---------------------------------------------------------------------------
// workspace arena: grow-only named device buffers owned by a handle
// ---------------------------------------------------------------------------
struct Buffer {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// HIP-event stage timers on the handle's stream (off unless enabled)
struct Profiler {
    bool on = false;
    double ms[ELM_STAGE_COUNT] = {};
    int64_t cnt[ELM_STAGE_COUNT] = {};
    struct Pending {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    hipEvent_t take();
    void resolve();  // synchronises on the recorded events
    void release();
};

struct StageScope {
    Profiler* p;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageScope(Profiler* prof, int st, hipStream_t stream);
    ~StageScope();
};

struct Workspace {
    std::vector<std::pair<std::string, Buffer>> bufs;
    std::vector<std::string> tables;  // buffers holding an uploaded constant table
    // instantiated HIP graphs of fixed launch sequences, by a key naming
    // everything their kernel arguments depend on (the most recent 32)
    std::vector<std::pair<std::string, hipGraphExec_t>> graphs;
    // the autotuners' table (elm_tune_entry rows): choices by kind, dtype and
    // the power-of-two buckets of the Gram's order and reduction length
    std::vector<elm_tune_entry> tune;
    Profiler* prof = nullptr;
    // HIP graphs captured and launched through this workspace, and host
    // synchronisations of the batched path's shared launches (counters)
    int64_t graph_captures = 0, graph_launches = 0, host_syncs = 0;
    void* get(const std::string& name, size_t bytes);
    void release();
    static int bucket(int64_t x) {  // ceil(log2 x), -1 for "any"
        if (x <= 0) return -1;
        int b = 0;
        while (((int64_t)1 << b) < x) ++b;
        return b;
    }
    // the tuned value for (kind, dtype, order n, length k), 0 if none
    int find_tune(int kind, int dt, int64_t n, int64_t k) const {
        const int nb = bucket(n), kb = bucket(k);
        for (const auto& t : tune)
            if (t.kind == kind && t.dtype == dt && t.n_log2 == nb && t.k_log2 == kb) return t.value;
        return 0;
    }
    void put_tune(int kind, int dt, int64_t n, int64_t k, int value) {
        const int nb = bucket(n), kb = bucket(k);
        for (auto& t : tune)
            if (t.kind == kind && t.dtype == dt && t.n_log2 == nb && t.k_log2 == kb) {
                t.value = value;
                return;
            }
        tune.push_back(elm_tune_entry{kind, dt, nb, kb, value});
    }
    // residual evaluations the last grouped refinement of a shape needed
    std::vector<std::pair<std::string, int>> iters;
    int find_iters(const std::string& key) const {
        for (const auto& x : iters)
            if (x.first == key) return x.second;
        return 1 << 20;
    }
    void put_iters(const std::string& key, int n) {
        for (auto& x : iters)
            if (x.first == key) {
                x.second = n;
                return;
            }
        if (iters.size() >= 64) iters.erase(iters.begin());
        iters.push_back({key, n});
    }
    hipGraphExec_t find_graph(const std::string& key) const {
        for (const auto& g : graphs)
            if (g.first == key) return g.second;
        return nullptr;
    }
    void put_graph(const std::string& key, hipGraphExec_t g) {
        if (graphs.size() >= 32) {
            (void)hipGraphExecDestroy(graphs.front().second);
            graphs.erase(graphs.begin());
        }
        graphs.push_back({key, g});
    }
    bool has_table(const std::string& name) const {
        for (const auto& t : tables)
            if (t == name) return true;
        return false;
    }
};

}  // namespace elm

namespace elm {
// Independent trainings of a batch run concurrently on this many streams by
// default (more than the runtime's four hardware queues per process: the
// streams also hide each other's host synchronisations).
constexpr int BATCH_WORKERS = 8;
// Grams of at least this order try the certified full-rank path first: from
// order ~48 up its blocked factorisation beats the n dependent greedy steps
// (0.07 against 0.24 ms at 64, 1.6 against 12.2 ms at 2000); below, the two
// are within launch overheads of each other
constexpr int64_t FULL_RANK_MIN_ORDER = 64;
// device memory for the Grams and factorisation scratch of one group of a
// batched training (larger batches run group after group)
constexpr size_t BATCH_GROUP_BYTES = (size_t)16 << 30;
}  // namespace elm

struct elm_handle {
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cu = 256;
    elm::Workspace ws;
    elm::Profiler prof;
    std::string last_error;
    // batched training: worker handles, each on a stream of its own (created
    // on first use, kept for reuse of their workspaces)
    std::vector<elm_handle*> workers;
    bool owns_stream = false;
    // second stream and its two ordering events, for work that overlaps the
    // handle's stream inside one call (created on first use)
    hipStream_t side = nullptr;
    // the stream of a batch's shared launches (created on first use)
    hipStream_t batch_stream = nullptr;
    hipEvent_t side_ev[2] = {nullptr, nullptr};
    // tuning options (elm_set_option)
    int64_t full_rank_min_order = elm::FULL_RANK_MIN_ORDER;
    int batch_workers = elm::BATCH_WORKERS;
    // counters of the last elm_train_batched call (elm_batch_get_report)
    elm_batch_report batch_report{};
};

struct elm_factor {
    int64_t N = 0, L = 0;     // shape of H
    int64_t n = 0;            // order of the Gram: min(N, L)
    int64_t r = 0;            // rank
    bool transposed = false;  // the Gram is H H^T (N < L)
    double tau = 0;           // absolute stopping threshold of the pivoted Cholesky
    // rank-decision diagnostics (host copies)
    elm_dtype gram_dtype = ELM_F64;  // element type the Gram was formed from
    double max_diag = 0, last_pivot = 0, first_rejected = 0;
    double noise_floor = 0;   // absolute rounding-noise scale of the Schur diagonals
    bool reliable = true;
    // 1: rank n by the certificate, identity order; 2: duplicated nodes set
    // aside, the distinct ones certified (rank = their count)
    int certified_full_rank = 0;
    // device buffers: hipMalloc'd and owned by the factor, or, when pool is
    // set, named buffers of that workspace (a factor used only inside a call)
    elm::Workspace* pool = nullptr;
    // or, when arena is set, carved from a caller's device arena (256-byte
    // aligned pieces, arena_left bytes still free; nothing is freed with the factor)
    char* arena = nullptr;
    size_t arena_left = 0;
    int32_t* piv = nullptr;   // n: original index at each pivoted position
    double* R = nullptr;      // r x n, pivot order, ld n: [R11 R12]
    double* Rinv = nullptr;   // r x r, ld r: R11^-1 (upper triangular)
    double* K = nullptr;      // r x (n - r), ld n - r: K = R11^-1 R12
    double* Usinv = nullptr;  // q x q, ld q: Us^-1 where Us^T Us = I + K K^T (q = r)
                              // or I + K^T K (q = n - r, woodbury)
    double* RinvT = nullptr;  // transposes, so every product in the solves reads rows
    double* KT = nullptr;     // (n - r) x r
    double* UsinvT = nullptr;
    int64_t q = 0;
    bool woodbury = false;
    // set while the Cholesky of the Gram of G has not been checked yet
    const int* pd_flag = nullptr;
    int device = 0;
};

namespace elm {
// A device buffer of a factor: from the factor's pool when it has one, else
// hipMalloc'd (freed by free_factor_buffers).
inline void* factor_alloc(elm_factor* f, const char* name, size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (f->arena) {
        bytes = (bytes + 255) & ~(size_t)255;
        if (bytes > f->arena_left)
            throw Error{ELM_ERR_ALLOC, std::string("factor buffer '") + name + "' exceeds its arena"};
        void* p = f->arena;
        f->arena += bytes;
        f->arena_left -= bytes;
        return p;
    }
    if (f->pool) return f->pool->get(std::string("factor_") + name, bytes);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess)
        throw Error{ELM_ERR_ALLOC, std::string("factor buffer '") + name + "': hipMalloc of " +
                                       std::to_string(bytes) + " bytes failed"};
    return p;
}
}  // namespace elm

namespace elm {

// ---------------------------------------------------------------------------
// kernel launchers (each .hip file owns its kernels)
// ---------------------------------------------------------------------------

// hidden.hip: H = sigmoid(X W + b), sample-major H and/or node-major low-precision copy
// Hidden layer; with Zpart (FP64 inputs, T non-null, 1 <= m <= HIDDEN_Z_MAX_M)
// it also writes the per-row-tile partials of Z = H^T T: Zpart[t][j][c] for
// row tile t of hidden_row_tiles(N) (sum them in order for Z).
constexpr int HIDDEN_Z_MAX_M = 8;
void launch_hidden(hipStream_t s, elm_dtype dt, int64_t N, int64_t d, int64_t L, const void* X,
                   int64_t ldx, const void* W, int64_t ldw, const void* b, void* H, int64_t ldh,
                   void* Hlp, int64_t ldlp, elm_dtype lp_dt, const double* T = nullptr,
                   int64_t ldt = 0, int64_t m = 0, double* Zpart = nullptr);
int64_t hidden_row_tiles(int64_t N);

// gram.hip: M (n x n FP64, full symmetric, ld = ldm)
//   column Gram  M = H^T H  of sample-major FP64 H (N x L)
void launch_gram_f64_cols(hipStream_t s, int64_t N, int64_t L, const double* H, int64_t ldh,
                          double* M, int64_t ldm, Workspace& ws, int force_chunks = 0);
//   row Gram     M = H H^T  of sample-major FP64 H (N x L, N < L)
void launch_gram_f64_rows(hipStream_t s, int64_t N, int64_t L, const double* H, int64_t ldh,
                          double* M, int64_t ldm, Workspace& ws);
//   column Gram of a node-major low-precision copy (L x N): M = Hn Hn^T.
//   Returns the longest run of products accumulated in FP32 before the FP64
//   sum of the partial Grams.
//   force_splits > 0 fixes the number of K splits (the autotuner's candidates);
//   otherwise an ELM_GRAM_SPLITS override, the autotuner's choice for this
//   shape, or the default rule decides.
int64_t launch_gram_lp_nodes(hipStream_t s, elm_dtype dt, int64_t N, int64_t L, const void* Hn,
                             int64_t ldn, double* M, int64_t ldm, Workspace& ws,
                             int force_splits = 0);
//   the default rule's K splits for a 16-bit Gram of L nodes over N samples,
//   and K chunks for an FP32/FP64 Gram of order n over K products
int gram_default_splits(int64_t N, int64_t L);
int gram16_default_chunks(int dt, int64_t n, int64_t K);
//   the Gram of elm_gram with its partial tiles in a static device array of
//   GRAM_NOALLOC_SCRATCH_BYTES per GPU instead of the workspace (no device
//   allocation); K splits lowered until they fit, ELM_ERR_SHAPE if none does
constexpr size_t GRAM_NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
void launch_gram_noalloc(hipStream_t s, int device, elm_dtype dt, int64_t N, int64_t L, const void* H,
                         int64_t ldh, double* M, int64_t ldm);
//   device address of that array on `device` (which must be current), looked
//   up once per device
void* noalloc_scratch(int device);
//   *out = max_i M[i][i]  (NaN if any diagonal entry is NaN)
void launch_diag_max(hipStream_t s, int64_t n, const double* M, int64_t ldm, double* out);

// pchol.hip: greedy pivoted Cholesky of M (n x n FP64, full symmetric, ld = ldm).
// Writes piv (n), allocates *R_out = R (r x n in pivot order, ld n, by factor_alloc,
// NULL when r = 0) and returns r (synchronises the stream once).  stats_out
// (host, 3 doubles): last accepted pivot (+inf if r = 0), largest Schur
// diagonal at the stop (-inf if r = n), largest Gram diagonal.
int64_t pivoted_cholesky(hipStream_t s, int64_t n, const double* M, int64_t ldm, double tau,
                         int32_t* piv, double** R_out, double* stats_out, Workspace& ws,
                         elm_factor* f);
void launch_fill(hipStream_t s, double* p, int64_t count, double v);

// One factorisation of a group run by pivoted_cholesky_grouped.  In: n, the
// Gram M (n x n FP64, full symmetric, ld ldm) and the threshold tau.  Out:
// rank, stats (as stats_out above), bad (a non-finite Gram diagonal), piv
// (device, n entries: accepted pivots, then the rejected positions) and
// Rorig (device, n x n, ld n: row k of R with its columns by original
// index); both stay valid until the workspace's next grouped call.
struct PcholProblem {
    int64_t n = 0;
    const double* M = nullptr;
    int64_t ldm = 0;
    double tau = 0.0;
    int64_t rank = 0;
    double stats[3] = {0, 0, 0};
    bool bad = false;
    const int32_t* piv = nullptr;
    const double* Rorig = nullptr;
};
// Factorises every problem of the group with the same pivot rule and the
// same arithmetic as pivoted_cholesky, in shared launches (one per pivot
// step for all problems together); synchronises the stream once.
void pivoted_cholesky_grouped(hipStream_t s, std::vector<PcholProblem>& probs, Workspace& ws);
// R (r x n, ld ldr) = the first r rows of Rorig with columns in pivot order
void launch_gather_rows(hipStream_t s, int64_t r, int64_t n, const double* Rorig, int64_t ldro,
                        const int32_t* piv, double* R, int64_t ldr);

// Relative rounding-noise scale of the Schur diagonals of a Gram formed from
// H rounded to `dt` with `kc` products per FP32 partial sum (kc = 0: FP64
// accumulation), for a Gram of order n over K samples.  A column that is an
// exact combination of others in FP64 but not after rounding keeps a residual
// of about u/sqrt(3) of its norm (u the unit roundoff of dt), i.e. a Schur
// diagonal of u^2/3 of the largest diagonal; FP32 accumulation adds about
// sqrt(kc) 2^-24 per Gram entry.
inline double schur_noise_floor(elm_dtype dt, int64_t n, int64_t K, int64_t kc) {
    const double u = dt == ELM_BF16 ? std::ldexp(1.0, -8)
                   : dt == ELM_F16  ? std::ldexp(1.0, -11)
                   : dt == ELM_F32  ? std::ldexp(1.0, -24)
                                    : std::ldexp(1.0, -53);
    const double acc = kc > 0 ? std::sqrt((double)kc) * std::ldexp(1.0, -24)
                              : std::sqrt((double)K) * std::ldexp(1.0, -53);
    const double fp64 = (double)n * std::ldexp(1.0, -53);
    return u * u / 3.0 + acc + fp64;
}

// gemm.hip: C = alpha A B + beta C on FP64 MFMA, strided operands
//   A(i, k) = A[i a_rs + k a_cs], B(k, j) = B[k b_rs + j b_cs]; a batch of
//   equally shaped products at strides a_bs, b_bs, c_bs.  tri_a / tri_b: A /
//   B upper triangular (their zero blocks are skipped); upper_c: only the
//   upper triangle of C is needed; skip: device flag, nothing runs when set.
void gemm_f64(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
              int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs, int64_t b_cs, double beta,
              double* C, int64_t ldc);
void gemm_f64_batched(hipStream_t s, int64_t batch, int64_t M, int64_t N, int64_t K, double alpha,
                      const double* A, int64_t a_rs, int64_t a_cs, int64_t a_bs, const double* B,
                      int64_t b_rs, int64_t b_cs, int64_t b_bs, double beta, double* C, int64_t ldc,
                      int64_t c_bs, bool tri_a, bool tri_b, bool upper_c = false,
                      const int* skip = nullptr);

// chol.hip: certified full-rank path of the rank step.  Factorises M = U^T U
// without pivoting (blocked, U in *R_out by factor_alloc, n x n, ld n, zero
// below the diagonal) and returns false without a result as soon as a pivot
// is <= thr.  Synchronises the stream once.
bool unpivoted_cholesky(hipStream_t s, int64_t n, const double* M, int64_t ldm, double thr,
                        double** R_out, elm_factor* f, Workspace& ws, hipStream_t side = nullptr,
                        hipEvent_t ev_main = nullptr, hipEvent_t ev_side = nullptr);
// In-place blocked Cholesky A = U^T U of the upper triangle of A (n x n, ld
// lda; zero below the diagonal afterwards); flag (device) is set, and the
// remaining work skipped, at a pivot <= thr.  No synchronisation.
// side (optional, with events ev_main and ev_side): a second stream on which
// the part of each trailing update beyond the next group of block rows runs
// while that group is factored on s.
void cholesky_blocked(hipStream_t s, int64_t n, double* A, int64_t lda, double thr, int* flag,
                      Workspace& ws, hipStream_t side = nullptr, hipEvent_t ev_main = nullptr,
                      hipEvent_t ev_side = nullptr);
// q <= 128: A = U^T U in place (upper, zero below) and Ainv = U^-1 (q x q, ld
// ldi), one workgroup; flag set at a pivot <= thr.  No synchronisation.
void cholesky_inverse_small(hipStream_t s, int64_t q, double* A, int64_t lda, double* Ainv,
                            int64_t ldi, int* flag, double thr = 0.0);
// 1 / max_j sum_k X[j][k]^2 over the rows of an upper triangular n x n X (ld
// ldx); synchronises the stream once.
double inv_max_row_sumsq(hipStream_t s, int64_t n, const double* X, int64_t ldx, Workspace& ws);
// piv[i] = i
void launch_iota(hipStream_t s, int64_t n, int32_t* piv);
// the diagonal of M into out (n values, device)
void launch_diag_copy(hipStream_t s, int64_t n, const double* M, int64_t ldm, double* out);
// Duplicated hidden nodes in a Gram M (n x n, upper triangle read, diagonal
// diag on the host): rep[j] = the lowest index whose Gram row equals row j
// bitwise (j itself when none).  Equal columns of H give bitwise-equal Gram
// rows; the candidates are the pairs of equal diagonal values whose cross
// term equals them too (two distinct columns with equal norms cannot show it:
// |M_ij| < M_ii by Cauchy-Schwarz unless they are parallel), and their whole
// rows are then compared (a synchronisation each, only when there are
// candidates).  Returns the number of columns j with rep[j] != j, or -1 when
// more than 65536 candidate pairs would have to be read.
int64_t duplicate_nodes(hipStream_t s, int64_t n, const double* M, int64_t ldm,
                        const std::vector<double>& diag, Workspace& ws, std::vector<int32_t>& rep);
// The unpivoted blocked Cholesky of the Gram of the distinct nodes (S: the j
// with rep[j] == j, ascending) stopping, like unpivoted_cholesky, at a pivot
// <= thr (false, nothing kept).  On success R_out = [R11 R12] (r x n, ld n,
// allocated for f) in the order S then the copies D (ascending), whose R12
// columns are their originals' columns of R11, and f->piv (allocated by the
// caller, n entries) holds that order.
bool dedup_cholesky(hipStream_t s, int64_t n, const double* M, int64_t ldm,
                    const std::vector<int32_t>& rep, double thr, double** R_out, elm_factor* f,
                    Workspace& ws, hipStream_t side, hipEvent_t ev_main, hipEvent_t ev_side);

// solve.hip: dense FP64 helpers for the factor and the pseudoinverse apply
//   C (M x m, ld ldc) = alpha A B + beta C for A (M x K, ld lda) and a thin B
//   (K x m, ld ldb, m <= 64); tri 1: A upper triangular (only k >= i read),
//   2: A lower triangular (k <= i), 0: dense
void rowprod(hipStream_t s, int64_t M, int64_t K, int64_t m, double alpha, const double* A, int64_t lda,
             int tri, const double* B, int64_t ldb, double beta, double* C, int64_t ldc);
//   B (Cn x R, ld R) = A^T for A (R x Cn, ld lda); returns B
double* transposed_copy(hipStream_t s, int64_t R, int64_t Cn, const double* A, int64_t lda, double* B);
//   dst[i][:] = src[idx[i]][:]  /  dst[idx[i]][:] = src[i][:]   (rows x cols)
void gather_rows(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds,
                 const int32_t* idx, double* dst, int64_t ldd);
void scatter_rows(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds,
                  const int32_t* idx, double* dst, int64_t ldd);
void zero_mat(hipStream_t s, int64_t rows, int64_t cols, double* A, int64_t lda);
//   X = U^-1 for upper-triangular U (r x r); X must not alias U
void trtri_upper(hipStream_t s, int64_t r, const double* U, int64_t ldu, double* X, int64_t ldx,
                 Workspace& ws);
// wait = false: no synchronisation; the positive-definiteness flag of the
// Gram of G is left in f->pd_flag (a workspace word) for the solve to read.
void build_factor_tail(hipStream_t s, elm_factor* f, Workspace& ws, bool wait = true);
void apply_pinv(hipStream_t s, const elm_factor* f, int64_t m, const double* rhs, int64_t ldr,
                const double* H64, int64_t ldh64, double* out, int64_t ldo, Workspace& ws);
// build_factor_tail for several factors (rank >= 1, buffers from factor_alloc)
// at once: every step one launch for all of them, with the same kernels and
// arithmetic per factor; Grams of G above order 128 take the blocked Cholesky
// one by one.  Rorig[p] (may be NULL): R of factor p is first gathered from it
// (n x n, ld n, columns by original index) through f->piv.  Returns per
// factor 1 when the Gram of G is not positive definite; synchronises once.
std::vector<int> build_factor_tails_grouped(hipStream_t s, const std::vector<elm_factor*>& fs,
                                            const std::vector<const double*>& Rorig, Workspace& ws);

// block.hip: the block form of Section 3 (eqs. 19-23) for a full-column-rank
// H split after `split` columns of the order piv (NULL: identity), from the
// FP64 Gram M (L x L, ld ldm) and Z = H^T T (L x m, ld ldz); beta (L x m, ld
// ldb).  Synchronises once; NOT_PSD when a pivot of A or D is <= thr.
void block_solve(hipStream_t s, int64_t L, int64_t m, int64_t split, const double* M, int64_t ldm,
                 const double* Z, int64_t ldz, const int32_t* piv, double thr, double* beta, int64_t ldb,
                 Workspace& ws);

// probe.hip: device ceilings (measurement only); each returns TFLOP/s or GB/s
double probe_mfma(hipStream_t s, elm_dtype dt, int shape, int random_ops, double* ms_out);
double probe_stream(hipStream_t s, const void* buf, int64_t bytes, double* ms_out);
double probe_dma(hipStream_t s, const void* buf, int64_t bytes, int resident, double* ms_out);

// grow.hip: the factor g of H' = [H Hn] (N x L2 FP64 sample-major, ld ldh, its
// first f->n columns the H of factor f: FP64 Gram, N >= L2) from f and the new
// Gram blocks, keeping f's accepted pivots first.  Returns false (g untouched
// beyond its scalar fields) when f's decision would not stand under the grown
// threshold.  Synchronises.
bool grow_factor(hipStream_t s, const elm_factor* f, int64_t N, int64_t L2, const double* H, int64_t ldh,
                 double tau_rel, elm_factor* g, Workspace& ws);

// refine.hip: streaming FP64 passes over sample-major H
//   E = T - H beta  (N x m)
//   (optionally also Y = H beta and the arg-max of each row of H beta)
void launch_residual(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H, int64_t ldh,
                     const double* T, int64_t ldt, const double* beta, int64_t ldb, double* E,
                     int64_t lde, double* Y = nullptr, int64_t ldy = 0, int32_t* labels = nullptr);
//   G = sum over chunks (in order) of part[chunk] (each L x m, row-major), and
//   *nrm2 = ||G||_F^2
void launch_partial_sum(hipStream_t s, int64_t L, int64_t m, int64_t nchunk, const double* part,
                        double* G, int64_t ldg, double* nrm2, Workspace& ws);
//   G = H^T E  (L x m), deterministic two-stage reduction; also writes ||G||_F^2 to *nrm2
void launch_ht_times(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H, int64_t ldh,
                     const double* E, int64_t lde, double* G, int64_t ldg, double* nrm2,
                     Workspace& ws);
//   Y = H beta and/or arg-max labels
void launch_hidden_output(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H,
                          int64_t ldh, const double* beta, int64_t ldb, double* Y, int64_t ldy,
                          int32_t* labels);
//   Y += X  (rows x cols, both row-major with their leading dimensions)
void launch_add_mat(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y,
                    int64_t ldy);
//   beta += delta, elementwise over L x m; prev (ld cols) receives beta before it
void launch_axpy_mat(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy, double* prev);

// ---------------------------------------------------------------------------
// Grouped launches over the problems of a batch.  Blocks [start[j],
// start[j + 1]) of a launch serve problem prob[j] (j < count); start (count +
// 1 entries) and prob are device arrays and blocks = start[count] < 2^31.
// Each block runs the single-problem kernel's body with its problem's
// arguments and its block index within that problem, so a grouped launch
// computes what the single-problem launches would, bit for bit.
// ---------------------------------------------------------------------------
struct GroupSched {
    const int32_t* start = nullptr;
    const int32_t* prob = nullptr;
    int count = 0;
    int64_t blocks = 0;
    // optional device flags by descriptor index: the blocks of a problem whose
    // flag is 0 return at once (refinement steps decided on the device)
    const int32_t* live = nullptr;
};
// the problem of this block (a descriptor index) and its block index within it
__device__ inline int group_problem(const GroupSched& g, int64_t& local) {
    const int32_t b = (int32_t)blockIdx.x;
    int lo = 0, hi = g.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g.start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    local = b - g.start[lo];
    return g.prob[lo];
}
__device__ inline bool group_live(const GroupSched& g, int j) { return g.live == nullptr || g.live[j] != 0; }

// A sequence of grouped launches: add() copies one launch's descriptors and
// schedule (problems with no blocks left out) into a host blob, call() inserts
// host-issued work; run() uploads the blob in one copy and issues everything
// in order on one stream (the blob stays valid until the workspace buffer
// `name` is requested again).
struct GroupProgram {
    typedef std::function<void(hipStream_t s, const void* desc, const GroupSched& g)> LaunchFn;
    struct Launch {
        size_t doff = 0, soff = 0;
        int count = 0;
        int64_t blocks = 0;
        LaunchFn fn;
        std::function<void()> call;
    };
    std::vector<char> blob;
    std::vector<Launch> launches;
    static size_t al(size_t b) { return (b + 255) & ~(size_t)255; }
    template <class D>
    void add(const std::vector<D>& descs, const std::vector<int64_t>& nblk, LaunchFn fn) {
        std::vector<int32_t> st, pr;
        int64_t tot = 0;
        for (size_t j = 0; j < descs.size(); ++j) {
            if (nblk[j] <= 0) continue;
            st.push_back((int32_t)tot);
            pr.push_back((int32_t)j);
            tot += nblk[j];
            if (tot >= INT32_MAX) throw Error{ELM_ERR_UNSUPPORTED, "grouped launch too large"};
        }
        if (pr.empty()) return;
        st.push_back((int32_t)tot);
        Launch l;
        l.count = (int)pr.size();
        l.blocks = tot;
        l.fn = std::move(fn);
        l.doff = al(blob.size());
        blob.resize(l.doff + descs.size() * sizeof(D));
        std::memcpy(blob.data() + l.doff, descs.data(), descs.size() * sizeof(D));
        l.soff = al(blob.size());
        blob.resize(l.soff + (st.size() + pr.size()) * sizeof(int32_t));
        std::memcpy(blob.data() + l.soff, st.data(), st.size() * sizeof(int32_t));
        std::memcpy(blob.data() + l.soff + st.size() * sizeof(int32_t), pr.data(),
                    pr.size() * sizeof(int32_t));
        launches.push_back(std::move(l));
    }
    void call(std::function<void()> f) {
        Launch l;
        l.call = std::move(f);
        launches.push_back(std::move(l));
    }
    void run(hipStream_t s, Workspace& ws, const char* name) {
        char* dev = blob.empty() ? nullptr : (char*)ws.get(name, blob.size());
        if (dev) {
            const hipError_t e = hipMemcpyAsync(dev, blob.data(), blob.size(), hipMemcpyHostToDevice, s);
            if (e != hipSuccess) throw Error{ELM_ERR_HIP, std::string("grouped program upload: ") +
                                                              hipGetErrorString(e)};
        }
        for (const Launch& l : launches) {
            if (l.call) {
                l.call();
                continue;
            }
            GroupSched g;
            g.start = (const int32_t*)(dev + l.soff);
            g.prob = g.start + l.count + 1;
            g.count = l.count;
            g.blocks = l.blocks;
            l.fn(s, dev + l.doff, g);
        }
    }
};

// gemm.hip, grouped: one (batched) product of gemm_f64_batched
struct GemmDesc {
    int64_t M = 0, N = 0, K = 0, batch = 0;
    double alpha = 1.0, beta = 0.0;
    const double* A = nullptr;
    int64_t a_rs = 0, a_cs = 0, a_bs = 0;
    const double* B = nullptr;
    int64_t b_rs = 0, b_cs = 0, b_bs = 0;
    double* C = nullptr;
    int64_t ldc = 0, c_bs = 0;
    int tri_a = 0, tri_b = 0;
};
// the tile gemm_f64_batched takes for this shape (128 or 64); the result does
// not depend on it (every tile sums k in the same order, and the products a
// triangular operand skips are exact zeros)
int gemm_tile(const GemmDesc& q);
int64_t gemm_group_blocks(const GemmDesc& q, int ts);
void launch_gemm_grouped(hipStream_t s, int ts, const GemmDesc* d, const GroupSched& g);

// solve.hip / chol.hip, grouped: one matrix step of a factor tail
struct MatDesc {
    int64_t rows = 0, cols = 0;
    const double* src = nullptr;
    int64_t lds = 0;
    double* dst = nullptr;
    int64_t ldd = 0;
    const int32_t* idx = nullptr;
    double* aux = nullptr;
    int64_t lda = 0;
    int* flag = nullptr;
};
enum class MatOp {
    ZERO,          // dst (rows x cols) = 0
    TRANSPOSE,     // dst (cols x rows) = src^T
    ADD_IDENTITY,  // dst[i][i] += 1, i < rows
    GATHER_COLS,   // dst[i][j] = src[i][idx[j]]
    TRTRI_LEAF,    // the leaf diagonal blocks of dst = src^-1 (src upper triangular, rows x rows)
    CHOL_INV_SMALL // dst (rows <= 128) = U^T U in place, aux = U^-1 (ld lda), *flag at a pivot <= 0
};
int64_t mat_group_blocks(MatOp op, const MatDesc& q);
void launch_mat_grouped(hipStream_t s, MatOp op, const MatDesc* d, const GroupSched& g);
void launch_chol_inv_small_grouped(hipStream_t s, const MatDesc* d, const GroupSched& g);

// hidden.hip, grouped: one problem's hidden layer (FP64 inputs), as launch_hidden
struct HiddenDesc {
    int64_t N = 0, d = 0, L = 0;
    const double* X = nullptr;
    int64_t ldx = 0;
    const double* W = nullptr;
    int64_t ldw = 0;
    const double* b = nullptr;
    double* H = nullptr;
    int64_t ldh = 0;
    void* Hlp = nullptr;
    int64_t ldlp = 0;
    elm_dtype lp_dt = ELM_F64;
    const double* T = nullptr;
    int64_t ldt = 0;
    int m = 0;
    double* Zp = nullptr;
};
int64_t hidden_group_blocks(const HiddenDesc& q);
void launch_hidden_grouped(hipStream_t s, const HiddenDesc* d, const GroupSched& g);

// gram.hip, grouped: one problem's column Gram M (L x L) as the single launch
// computes it (16-bit or FP32 node-major H, or FP64 sample-major H)
enum GramKind { GRAM_BF16 = 0, GRAM_F16 = 1, GRAM_F32 = 2, GRAM_F64 = 3 };
struct GramDesc {
    int kind = 0;
    int64_t n = 0, K = 0, kc_len = 0, ntile = 0, nsplit = 0, nblocks = 0;
    const void* A = nullptr;  // H: node-major (ld N) or, for FP64, sample-major
    int64_t ld = 0;
    void* part = nullptr;     // the partial tiles (gram_group_plan's bytes)
    const int4* work = nullptr;
    double* M = nullptr;
    int64_t ldm = 0;
    double* dmax = nullptr;   // stage 2: the largest diagonal entry (NaN if any is NaN or Inf)
};
// Plans q for the Gram the single-problem launch of this dtype takes: kind,
// tiles, splits, chunk length and (16-bit) the work table, uploaded once per
// workspace.  Returns the bytes of its partials; *kc_out: the products per
// FP32 partial sum (the single launch's return value).
size_t gram_group_plan(hipStream_t s, elm_dtype dt, int64_t N, int64_t L, GramDesc& q,
                       Workspace& ws, int64_t* kc_out);
// stage 0: the partial products, 1: their FP64 sum into M, 2: the diagonal maximum
int64_t gram_group_blocks(int stage, const GramDesc& q);
void launch_gram_grouped(hipStream_t s, int stage, int kind, const GramDesc* d, const GroupSched& g);

// refine.hip, grouped: launch_partial_sum of one problem (Z = sum of its
// row-tile partials and ||Z||_F^2)
struct PsumDesc {
    int64_t L = 0, m = 0, nchunk = 0;
    const double* part = nullptr;  // nchunk x (L x m)
    double* part2 = nullptr;       // psum_part2_doubles(L, m, nchunk) (when nchunk > 128)
    double* G = nullptr;           // L x m, ld m
    double* sq = nullptr;          // refine_sq_doubles(L, m)
    double* nrm2 = nullptr;
};
size_t psum_part2_doubles(int64_t L, int64_t m, int64_t nchunk);
// group sums (problems with nchunk > 128), the column sums and squares, the total
void launch_partial_sum_grouped(hipStream_t s, int stage, const PsumDesc* d, const GroupSched& g);
int64_t partial_sum_group_blocks(int stage, const PsumDesc& q);

// refine.hip, grouped: one problem's refinement buffers (m <= 16)
struct RefineDesc {
    int64_t N = 0, L = 0;
    int m = 0;
    const double* H = nullptr;  // N x L sample-major FP64
    int64_t ldh = 0;
    const double* T = nullptr;  // N x m
    int64_t ldt = 0;
    double* beta = nullptr;     // L x m
    int64_t ldbeta = 0;
    double* E = nullptr;        // N x m, ld m: T - H beta
    double* part = nullptr;     // refine_part_doubles(N, L, m): column partials of H^T E
    double* G = nullptr;        // L x m, ld m: H^T E
    double* sq = nullptr;       // refine_sq_doubles(L, m)
    double* g2 = nullptr;       // ||G||_F^2
    double* D = nullptr;        // L x m, ld m: the correction added to beta
    double* prev = nullptr;     // L x m, ld m: beta before the last correction
    const double* z2 = nullptr; // ||H^T T||_F^2
};
// Refinement loop state of one problem, kept and decided on the device: the
// rules of elm_pinv_solve (stop at ir_tol after at least one correction, at
// ir_max_iter, or when a correction did not lower the residual).  A
// correction after which the residual exceeds IR_RISE times the previous one
// has diverged and is taken back.  Near the rounding floor the residuals of
// successive iterates differ by small factors at random, and there a
// correction that does not lower the residual is kept: the first corrections
// after an FP64 factor of an ill-conditioned Gram remove a forward error of
// about kappa^2 eps that the residual (already at its floor) does not show.
constexpr double IR_RISE = 4.0;
struct IrCtl {
    int32_t active = 0;    // still iterating
    int32_t it = 0;        // corrections kept
    int32_t evals = 0;     // residuals evaluated
    double prev = 0.0;     // residual before the last correction
    double res = 0.0;      // residual of the current beta
    double hist[32] = {};  // residual at each evaluation
};
// c[j] = iterating, flags cleared (P problems)
void launch_ir_init(hipStream_t s, int P, IrCtl* c, int32_t* active, int32_t* rollback);
// after the residual of every active problem: its decision.  g2 and z2 come
// from d[j] (descriptor j of P); active[j] / rollback[j] gate the next
// launches (rollback: this correction is taken back); *any = 1 while some
// problem is still iterating.
void launch_ir_decide(hipStream_t s, int P, IrCtl* c, const RefineDesc* d, int32_t* active,
                      int32_t* rollback, int32_t* any, double ir_tol, int ir_max_iter);
// beta = prev for the problems whose flag in g.live is set
void launch_restore_grouped(hipStream_t s, const RefineDesc* d, const GroupSched& g);
enum class RefinePass {
    ROWS_DOT,   // E = T - H beta
    COLS_DOT,   // part = column-chunk partials of H^T E
    HT_REDUCE,  // G = sum of the partials, per-block sums of squares
    SUM,        // g2 = ||G||_F^2
    AXPY        // prev = beta, beta += D
};
// blocks of problem q in a launch whose largest m is maxm
int64_t refine_group_blocks(RefinePass pass, const RefineDesc& q, int maxm);
size_t refine_part_doubles(int64_t N, int64_t L, int64_t m);
size_t refine_sq_doubles(int64_t L, int64_t m);
// maxm: the largest m of the scheduled problems
void launch_refine_grouped(hipStream_t s, RefinePass pass, const RefineDesc* d, const GroupSched& g,
                           int maxm);

// solve.hip, grouped: C = alpha A B + beta C with thin B (the apply's products)
struct RowprodDesc {
    int64_t M = 0, K = 0;
    int m = 0, tri = 0;  // tri 1: A upper triangular (k >= i), 2: lower (k <= i)
    double alpha = 1.0, beta = 0.0;
    const double* A = nullptr;
    int64_t lda = 0;
    const double* B = nullptr;
    int64_t ldb = 0;
    double* C = nullptr;
    int64_t ldc = 0;
};
//   row copies through an index: gather dst[i] = src[idx[i]], scatter dst[idx[i]] = src[i]
struct CopyRowsDesc {
    int64_t rows = 0, cols = 0;
    const double* src = nullptr;
    int64_t lds = 0;
    const int32_t* idx = nullptr;
    double* dst = nullptr;
    int64_t ldd = 0;
};
int64_t rowprod_group_blocks(const RowprodDesc& q, int maxm);
int64_t copy_rows_group_blocks(const CopyRowsDesc& q);
void launch_rowprod_grouped(hipStream_t s, const RowprodDesc* d, const GroupSched& g, int maxm);
void launch_copy_rows_grouped(hipStream_t s, bool scatter, const CopyRowsDesc* d, const GroupSched& g);

// predict.hip
void launch_predict(hipStream_t s, elm_dtype dt, int64_t N, int64_t d, int64_t L, int64_t m,
                    const void* X, int64_t ldx, const void* W, int64_t ldw, const void* b,
                    const double* beta, int64_t ldbeta, void* Y, int64_t ldy, int32_t* labels,
                    Workspace& ws);

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
// leading dimension of an internal node-major low-precision copy of H: a
// multiple of 64 elements, so that the 16-bit Gram's 64-sample row segments
// are whole 128-byte cache lines
inline int64_t lp_ld(int64_t N) { return cdiv(N, 64) * 64; }

}  // namespace elm
