// Certified full-rank path of the rank step (Section 3, eq. 6; algorithm
// step 4), for Grams of large order.
//
// The greedy pivoted Cholesky accepts every position of an n x n Gram M
// exactly when its smallest pivot exceeds tau.  Its pivots never increase
// (each step only lowers the remaining Schur diagonals), and its last pivot
// is the Schur complement of the last remaining index j with respect to all
// the others, 1 / (M^-1)_jj.  So every greedy pivot is at least
//   lambda = 1 / max_j (M^-1)_jj = 1 / max_j || row j of U^-1 ||^2
// for any Cholesky factor M = U^T U, pivoted or not.  When lambda clears the
// threshold with a margin, the greedy rule keeps all n positions and the rank
// is n without running the n sequential pivot steps: an unpivoted blocked
// Cholesky (MFMA products) and the row norms of U^-1 (which the solves need
// anyway) decide it.  Otherwise the caller runs the greedy factorisation.
//
// Organisation, per diagonal block of CB positions:
//   strip         the block rows take the updates of the earlier block rows
//                 of their group of GB rows            (FP64 MFMA GEMM)
//   potrf_block   one workgroup: the block's Cholesky factor (held in
//                 registers), written to U, then its inverse (in LDS), written
//                 to W
//   copy          the block rows right of the diagonal block into T
//   product       U12 = W^T T                           (FP64 MFMA GEMM)
// and per group: S -= U_g^T U_g on the trailing matrix's upper tiles, with
// U_g the group's GB rows (FP64 MFMA GEMM, GB deep).
// A block that meets a pivot <= thr sets a device flag, and every later
// kernel returns at once.
#include "elm_internal.h"

#include <algorithm>
#include <cmath>

namespace elm {
namespace {

constexpr int CB = 128;    // diagonal block
constexpr int GB = 4 * CB; // block rows per trailing update
constexpr int CPT = 1024;  // threads of the block kernel

__global__ void clear_flag_kernel(int* flag) {
    if (threadIdx.x == 0) *flag = 0;
}

// U = upper triangle of M (diagonal included), zero below
__global__ void copy_upper_kernel(int64_t n, const double* __restrict__ M, int64_t ldm,
                                  double* __restrict__ U, int64_t ldu) {
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
             c += (int64_t)gridDim.x * blockDim.x)
            U[i * ldu + c] = c >= i ? M[i * ldm + c] : 0.0;
}

// zero below the diagonal of U
__global__ void zero_lower_kernel(int64_t n, double* __restrict__ U, int64_t ldu) {
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y)
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < i;
             c += (int64_t)gridDim.x * blockDim.x)
            U[i * ldu + c] = 0.0;
}

// lane l's value of x, read by every lane of the wave (l wave-uniform)
__device__ __forceinline__ double readlane_f64(double x, int l) {
    const unsigned long long v = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
    return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Steps j = 32 JH .. 32 JH + 31 of the block Cholesky below (JH: the slice of
// the pivot rows, a compile-time index into the thread's registers).
// Returns true when a pivot is <= thr (every thread alike).
template <int JH>
__device__ __forceinline__ bool potrf_slice(double (&u)[4][4], double (*rowb)[CB], int* stop, int nb,
                                            double thr, int tx, int ty) {
    for (int jl = 0; jl < 32; ++jl) {
        const int j = 32 * JH + jl, pb = j & 1;
        if (j >= nb) return false;
        if (ty == jl) {
            // the pivot (j, j): slot (JH, JH) of lane 32 (jl % 2) + jl of this wave
            const double d = readlane_f64(u[JH][JH], 32 * (jl & 1) + jl);
            const bool ok = d > thr;
            const double dd = ok ? d : 1.0;
            // 1 / sqrt(dd): the hardware estimate (about 23 bits) and two
            // Newton-Raphson steps y <- y (3 - dd y^2) / 2, a short dependent
            // chain on the step's critical path; the root is dd y
            const double hd = 0.5 * dd;
            double y = __builtin_amdgcn_rsq(dd);
            y = y * fma(-hd, y * y, 1.5);
            y = y * fma(-hd, y * y, 1.5);
            const double rj = dd * y, inv = y;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int c = tx + 32 * b;
                const double x = c > j ? u[JH][b] * inv : (c == j ? rj : 0.0);
                rowb[pb][c] = x;
                u[JH][b] = x;
            }
            if (tx == 0) stop[pb] = ok ? 0 : 1;
        }
        __syncthreads();
        if (stop[pb]) return true;  // the same value for every thread
#pragma unroll
        for (int a = JH; a < 4; ++a) {  // slices a < JH hold final rows only
            if (a == JH && jl == 31) continue;  // nor does slice JH after its last step
            const int i = ty + 32 * a;
            const double ri = rowb[pb][i];
#pragma unroll
            for (int b = a; b < 4; ++b) {  // b < a: below the diagonal
                const int c = tx + 32 * b;
                if (i > j && c >= i) u[a][b] -= ri * rowb[pb][c];
            }
        }
    }
    return false;
}

// The CB x CB block lives in registers: thread (ty, tx) of a 32 x 32 grid
// holds the 4 x 4 elements (ty + 32 a, tx + 32 b), so the 32 owners of a row
// are one half of a wave.  Step j: the owners of row j read its pivot from
// the diagonal owner's lane (readlane), scale the row and publish it in LDS
// (with the stop decision); after one block barrier every thread applies
// the row to its elements.  Row and pivot buffers alternate between steps,
// so one barrier per step suffices.  A step's work is issue-bound, so the
// element slices a step cannot change are skipped by block-uniform tests:
// slices below the diagonal (b < a) and slices whose rows are all final.
// The inverse is then formed in LDS by recursive doubling (log2 CB levels of
// two small products each) rather than by CB more dependent steps.
__device__ __forceinline__ void potrf_block_body(double* __restrict__ U, int64_t ldu, int64_t k0,
                                                 int nb, double thr, double* __restrict__ W,
                                                 int64_t ldw, int* flag) {
    static_assert(CB == 128 && CPT == 1024, "4 x 4 elements per thread of a 32 x 32 grid");
    __shared__ double rowb[2][CB];
    __shared__ int stop[2];
    __shared__ double Us[CB][CB + 1];  // the factor, for the inverse's columns
    if (*flag) return;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    double u[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 32 * a, c = tx + 32 * b;
            u[a][b] = (i < nb && c < nb && c >= i) ? U[(k0 + i) * ldu + k0 + c] : 0.0;
        }
    // right-looking Cholesky: row j scaled by the root of its pivot, then
    // u[i][c] -= U[j][i] U[j][c] for j < i <= c
    if (potrf_slice<0>(u, rowb, stop, nb, thr, tx, ty) || potrf_slice<1>(u, rowb, stop, nb, thr, tx, ty) ||
        potrf_slice<2>(u, rowb, stop, nb, thr, tx, ty) || potrf_slice<3>(u, rowb, stop, nb, thr, tx, ty)) {
        if (threadIdx.x == 0) *flag = 1;  // the block leaves together
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 32 * a, c = tx + 32 * b;
            const double x = c >= i ? u[a][b] : 0.0;
            Us[i][c] = x;
            if (i < nb && c < nb) U[(k0 + i) * ldu + k0 + c] = x;
        }
    // W = U^-1 in place in Us by recursive doubling: first the inverted
    // diagonal, then for s = 1, 2, ..., CB / 2 each pair of inverted s x s
    // diagonal blocks A^-1, C^-1 and the block B of U between them give the
    // inverse's block -A^-1 (B C^-1): two products whose entries are staged in
    // registers across a barrier before they overwrite B.  Each entry is a sum
    // over k in increasing order (the triangular factors' zeros bound k).  Rows
    // past nb carry an identity, so they add exact zeros.
    __syncthreads();  // Us complete
    if (threadIdx.x < CB) {
        const int i = threadIdx.x;
        Us[i][i] = i < nb ? 1.0 / Us[i][i] : 1.0;
    }
    __syncthreads();
    for (int s = 1; s < CB; s *= 2) {
        const int E = s >= 16 ? s / 16 : 1;  // entries per thread: a 1 x E row piece
        const int groups = s / E;            // row pieces per row
        const int t = threadIdx.x;
        const bool act = t < (CB / (2 * s)) * s * groups;  // pairs x rows x pieces
        const int pg = s * groups;
        const int i0 = act ? 2 * s * (t / pg) : 0, i = act ? (t % pg) / groups : 0;
        const int j0 = act ? (t % groups) * E : 0;   // first column of the piece within C
        const int ra = i0 + i, cb = i0 + s + j0;     // row in A, first column in C
        double acc[4];
        // T = B C^-1: row ra of B times columns cb .. cb + E - 1 of C^-1 (rows k <= column)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = 0.0;
        if (act)
            for (int k = 0; k < j0 + E; ++k) {
                const double bik = Us[ra][i0 + s + k];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e < E) acc[e] += bik * Us[i0 + s + k][cb + e];
            }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (act && e < E) Us[ra][cb + e] = acc[e];
        __syncthreads();
        // -A^-1 T: row i of A^-1 (columns k >= i) times the same columns of T
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[e] = 0.0;
        if (act)
            for (int k = i; k < s; ++k) {
                const double aik = Us[ra][i0 + k];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (e < E) acc[e] += aik * Us[i0 + k][cb + e];
            }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (act && e < E) Us[ra][cb + e] = -acc[e];
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 32 * a, c = tx + 32 * b;
            if (i < nb && c < nb) W[i * ldw + c] = c >= i ? Us[i][c] : 0.0;
        }
}

__global__ __launch_bounds__(CPT) void potrf_block_kernel(double* __restrict__ U, int64_t ldu,
                                                          int64_t k0, int nb, double thr,
                                                          double* __restrict__ W, int64_t ldw,
                                                          int* flag) {
    potrf_block_body(U, ldu, k0, nb, thr, W, ldw, flag);
}

// one block per factor: dst (rows <= CB) factored in place, aux = its inverse
__global__ __launch_bounds__(CPT) void chol_inv_small_grouped(const MatDesc* __restrict__ d,
                                                              GroupSched g) {
    int64_t lb;
    const MatDesc& q = d[group_problem(g, lb)];
    potrf_block_body(q.dst, q.ldd, 0, (int)q.rows, 0.0, q.aux, q.lda, q.flag);
}

// T (nb x nc, ld nc) = U[k0 .. k0 + nb)[c0 .. c0 + nc)
__global__ void copy_rows_kernel(int nb, int64_t nc, const double* __restrict__ U, int64_t ldu,
                                 int64_t k0, int64_t c0, double* __restrict__ T, const int* flag) {
    if (*flag) return;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (c < nc && i < nb) T[i * nc + c] = U[(k0 + i) * ldu + c0 + c];
}

// out[j] = sum_{k >= j} X[j][k]^2, one block per row
__global__ __launch_bounds__(256) void row_sumsq_kernel(int64_t n, const double* __restrict__ X,
                                                        int64_t ldx, double* __restrict__ out) {
    __shared__ double part[4];
    for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
        double s = 0.0;
        for (int64_t k = j + threadIdx.x; k < n; k += 256) {
            const double x = X[j * ldx + k];
            s += x * x;
        }
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) out[j] = (part[0] + part[1]) + (part[2] + part[3]);
        __syncthreads();
    }
}

// *out = max of v[0 .. n) (NaN if any entry is NaN)
__global__ __launch_bounds__(1024) void max_kernel(int64_t n, const double* __restrict__ v,
                                                   double* __restrict__ out) {
    __shared__ double wm[16];
    double m = -INFINITY;
    bool nan = false;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const double x = v[i];
        if (x != x) nan = true;
        m = x > m ? x : m;
    }
    if (nan) m = NAN;
    for (int off = 32; off > 0; off >>= 1) {
        const double y = __shfl_xor(m, off);
        m = (m != m || y != y) ? NAN : (y > m ? y : m);
    }
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = wm[0];
        for (int w = 1; w < 16; ++w) r = (r != r || wm[w] != wm[w]) ? NAN : (wm[w] > r ? wm[w] : r);
        *out = r;
    }
}

__global__ void iota_kernel(int64_t n, int32_t* piv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) piv[i] = (int32_t)i;
}

}  // namespace

void cholesky_blocked(hipStream_t s, int64_t n, double* U, int64_t ldu, double thr, int* flag,
                      Workspace& ws, hipStream_t side, hipEvent_t ev_main, hipEvent_t ev_side) {
    const bool look = side && ev_main && ev_side;
    bool side_pending = false;
    double* W = (double*)ws.get("fr_W", (size_t)CB * CB * sizeof(double));
    double* T = (double*)ws.get("fr_T", (size_t)CB * n * sizeof(double));
    // Groups of GB block rows: inside a group each block row first takes the
    // updates of the group's earlier rows (left-looking, one product), so the
    // trailing matrix is updated once per group with a GB-row-deep product.
    for (int64_t g0 = 0; g0 < n; g0 += GB) {
        const int64_t g1 = std::min<int64_t>(g0 + GB, n);
        for (int64_t k0 = g0; k0 < g1; k0 += CB) {
            const int nb = (int)std::min<int64_t>(CB, n - k0);
            if (k0 > g0) {
                // rows k0 .. k0 + nb, columns k0 .. n  -=  U[g0 .. k0)[k0 ..]^T U[g0 .. k0)[k0 ..]
                const double* Ug = U + g0 * ldu + k0;
                gemm_f64_batched(s, 1, nb, n - k0, k0 - g0, -1.0, Ug, 1, ldu, 0, Ug, ldu, 1, 0, 1.0,
                                 U + k0 * ldu + k0, ldu, 0, false, false, true, flag);
            }
            potrf_block_kernel<<<1, CPT, 0, s>>>(U, ldu, k0, nb, thr, W, CB, flag);
            ELM_LAUNCH_CHECK();
            const int64_t c0 = k0 + nb, nc = n - c0;
            if (nc <= 0) break;
            copy_rows_kernel<<<dim3((unsigned)cdiv(nc, 256), (unsigned)nb), 256, 0, s>>>(nb, nc, U, ldu,
                                                                                       k0, c0, T, flag);
            ELM_LAUNCH_CHECK();
            // U12 = W^T T: A(i, k) = W[k][i]
            gemm_f64_batched(s, 1, nb, nc, nb, 1.0, W, 1, CB, 0, T, nc, 1, 0, 0.0, U + k0 * ldu + c0,
                             ldu, 0, false, false, false, flag);
        }
        if (g1 >= n) continue;
        if (!look) {
            // S -= U[g0 .. g1)[g1 ..]^T U[g0 .. g1)[g1 ..] on the upper tiles
            const double* Ug = U + g0 * ldu + g1;
            gemm_f64_batched(s, 1, n - g1, n - g1, g1 - g0, -1.0, Ug, 1, ldu, 0, Ug, ldu, 1, 0, 1.0,
                             U + g1 * ldu + g1, ldu, 0, false, false, true, flag);
            continue;
        }
        // Look-ahead: the next group's rows [g1, g2) now (after the previous
        // group's remote update, which also wrote them), the rows beyond g2
        // on the side stream, overlapping the next group's diagonal blocks.
        const int64_t g2 = std::min<int64_t>(g1 + GB, n);
        if (side_pending) ELM_HIP_TRY(hipStreamWaitEvent(s, ev_side, 0));
        const double* Ug = U + g0 * ldu + g1;
        gemm_f64_batched(s, 1, g2 - g1, n - g1, g1 - g0, -1.0, Ug, 1, ldu, 0, Ug, ldu, 1, 0, 1.0,
                         U + g1 * ldu + g1, ldu, 0, false, false, true, flag);
        if (g2 < n) {
            ELM_HIP_TRY(hipEventRecord(ev_main, s));
            ELM_HIP_TRY(hipStreamWaitEvent(side, ev_main, 0));
            const double* Ub = U + g0 * ldu + g2;
            gemm_f64_batched(side, 1, n - g2, n - g2, g1 - g0, -1.0, Ub, 1, ldu, 0, Ub, ldu, 1, 0, 1.0,
                             U + g2 * ldu + g2, ldu, 0, false, false, true, flag);
            ELM_HIP_TRY(hipEventRecord(ev_side, side));
            side_pending = true;
        }
    }
    if (side_pending) ELM_HIP_TRY(hipStreamWaitEvent(s, ev_side, 0));
    // the updates left values below the diagonal of the blocks that straddle
    // it; U must be zero there
    zero_lower_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)std::min<int64_t>(n, 65535)), 256, 0,
                        s>>>(n, U, ldu);
    ELM_LAUNCH_CHECK();
}

void launch_chol_inv_small_grouped(hipStream_t s, const MatDesc* d, const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    chol_inv_small_grouped<<<(unsigned)g.blocks, CPT, 0, s>>>(d, g);
    ELM_LAUNCH_CHECK();
}

void cholesky_inverse_small(hipStream_t s, int64_t q, double* A, int64_t lda, double* Ainv,
                            int64_t ldi, int* flag, double thr) {
    if (q <= 0) return;
    if (q > CB) throw Error{ELM_ERR_INVALID_ARG, "cholesky_inverse_small: order above 128"};
    potrf_block_kernel<<<1, CPT, 0, s>>>(A, lda, 0, (int)q, thr, Ainv, ldi, flag);
    ELM_LAUNCH_CHECK();
}

bool unpivoted_cholesky(hipStream_t s, int64_t n, const double* M, int64_t ldm, double thr,
                        double** R_out, elm_factor* f, Workspace& ws, hipStream_t side,
                        hipEvent_t ev_main, hipEvent_t ev_side) {
    *R_out = nullptr;
    double* U = (double*)factor_alloc(f, "R", (size_t)n * n * sizeof(double));
    int* flag = (int*)ws.get("fr_flag", sizeof(int));
    clear_flag_kernel<<<1, 64, 0, s>>>(flag);
    ELM_LAUNCH_CHECK();
    copy_upper_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)std::min<int64_t>(n, 65535)), 256, 0,
                        s>>>(n, M, ldm, U, n);
    ELM_LAUNCH_CHECK();
    cholesky_blocked(s, n, U, n, thr, flag, ws, side, ev_main, ev_side);
    int hflag = 0;
    ELM_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    if (hflag) {
        if (!f->pool) (void)hipFree(U);
        return false;
    }
    *R_out = U;
    return true;
}

double inv_max_row_sumsq(hipStream_t s, int64_t n, const double* X, int64_t ldx, Workspace& ws) {
    double* rows = (double*)ws.get("fr_rows", (size_t)n * sizeof(double));
    double* mx = (double*)ws.get("fr_max", sizeof(double));
    row_sumsq_kernel<<<(unsigned)std::min<int64_t>(n, 8192), 256, 0, s>>>(n, X, ldx, rows);
    ELM_LAUNCH_CHECK();
    max_kernel<<<1, 1024, 0, s>>>(n, rows, mx);
    ELM_LAUNCH_CHECK();
    double h = 0.0;
    ELM_HIP_TRY(hipMemcpyAsync(&h, mx, sizeof(double), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    return h > 0.0 ? 1.0 / h : 0.0;
}

void launch_iota(hipStream_t s, int64_t n, int32_t* piv) {
    if (n <= 0) return;
    iota_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(n, piv);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
