// From the rank step to beta (Section 3; eq. 7 and step 9 of the algorithm).
//
// With the pivoted factor P^T M P = R^T R, R = [R11 R12] (r x n):
//   F = H1 = H P[:, :r]  (the r independent columns),  F^T F = R11^T R11,
//   K = R11^-1 R12,  G = [I K] P^T,  G G^T = I + K K^T,
//   H^+ = G^T (G G^T)^-1 (F^T F)^-1 F^T.
// When N < L the same factorisation is taken of H^T (Gram H H^T) and
//   H^+ = F' (F'^T F')^-1 (G' G'^T)^-1 G'  with F' = H[piv[:r], :]^T.
//
// The factor keeps explicit inverses of the triangular factors (R11^-1 and
// the inverse Cholesky factor of I + K K^T, or of I + K^T K used through the
// Woodbury identity when n - r < r), so each application of H^+ is a short
// chain of matrix products on the FP64 MFMA.  The triangular inverse is built
// by recursive doubling of diagonal blocks:
//   [A B; 0 C]^-1 = [A^-1, -A^-1 B C^-1; 0, C^-1].
#include "elm_internal.h"

#include <algorithm>
#include <cstring>
#include <functional>

namespace elm {

namespace {

constexpr int LB = 64;  // leaf block of the triangular inverse

// invert the LB x LB (or smaller, last) diagonal blocks of upper-triangular U
__device__ __forceinline__ void trtri_leaf_body(int64_t bx, int64_t r, const double* __restrict__ U,
                                                int64_t ldu, double* __restrict__ X, int64_t ldx) {
    __shared__ double Us[LB][LB + 1];
    __shared__ double Xs[LB][LB + 1];
    const int64_t b0 = bx * LB;
    const int nb = (int)((r - b0) < LB ? (r - b0) : LB);
    const int j = threadIdx.x;
    for (int i = 0; i < nb; ++i)
        if (j < nb) Us[i][j] = U[(b0 + i) * ldu + b0 + j];
    __syncthreads();
    if (j < nb) {
        // column j of the inverse: X[j][j] = 1/U[j][j], back substitution upward
        for (int i = 0; i < nb; ++i) Xs[i][j] = 0.0;
        Xs[j][j] = 1.0 / Us[j][j];
        for (int i = j - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= j; ++k) s += Us[i][k] * Xs[k][j];
            Xs[i][j] = -s / Us[i][i];
        }
    }
    __syncthreads();
    for (int i = 0; i < nb; ++i)
        if (j < nb) X[(b0 + i) * ldx + b0 + j] = Xs[i][j];
}

__global__ __launch_bounds__(LB) void trtri_leaf_kernel(int64_t r, const double* __restrict__ U,
                                                        int64_t ldu, double* __restrict__ X,
                                                        int64_t ldx) {
    trtri_leaf_body(blockIdx.x, r, U, ldu, X, ldx);
}

__global__ void add_identity_kernel(int64_t q, double* A, int64_t lda) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < q) A[i * lda + i] += 1.0;
}

// dst[i][c] = src[idx[i]][c]
__global__ void gather_rows_kernel(int64_t rows, int64_t cols, const double* __restrict__ src,
                                   int64_t lds, const int32_t* __restrict__ idx,
                                   double* __restrict__ dst, int64_t ldd) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (c < cols && i < rows) dst[i * ldd + c] = src[(int64_t)idx[i] * lds + c];
}

// dst[idx[i]][c] = src[i][c]
__global__ void scatter_rows_kernel(int64_t rows, int64_t cols, const double* __restrict__ src,
                                    int64_t lds, const int32_t* __restrict__ idx,
                                    double* __restrict__ dst, int64_t ldd) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (c < cols && i < rows) dst[(int64_t)idx[i] * ldd + c] = src[i * lds + c];
}

__global__ void zero_mat_kernel(int64_t rows, int64_t cols, double* __restrict__ A, int64_t lda) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (c < cols && i < rows) A[i * lda + c] = 0.0;
}

// C[i][c] = alpha * sum_k A[i][k] B[k][c] + beta * C[i][c] for thin B (m <= MM
// columns): a wave takes RP rows (so that each B value read serves RP rows),
// lane l the columns k = l (mod 64) of every row, fixed-order lane reduction.
// tri restricts k to the nonzero part of a triangular A (1: k >= i, 2:
// k <= i); a row's columns outside its range are masked, so its lane sums,
// and by the halving exchange its whole sum, do not depend on which rows
// share its wave (the batch's launches may take another MM than a single
// problem's).
template <int MM>
struct Rowprod {
    static constexpr int RP = MM <= 16 ? 4 : 1;  // rows per wave
    static constexpr int RB = 4 * RP;             // rows per block
};

template <int MM>
__device__ __forceinline__ void rowprod_body(int64_t bx, int64_t M, int64_t K, int m, double alpha,
                                    const double* __restrict__ A, int64_t lda, int tri,
                                    const double* __restrict__ B, int64_t ldb, double beta,
                                    double* C, int64_t ldc) {
    constexpr int RP = Rowprod<MM>::RP;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t i0 = (bx * 4 + wave) * RP;
    if (i0 >= M) return;
    // the wave's columns: the union of its rows' ranges, from a multiple of 64
    int64_t kb = 0, ke = K;
    if (tri == 1) kb = i0 & ~(int64_t)63;
    if (tri == 2) ke = min(K, min(i0 + RP, M));
    double acc[RP][MM];
    const double* __restrict__ arow[RP];
    int64_t klo[RP], khi[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
#pragma unroll
        for (int c = 0; c < MM; ++c) acc[r][c] = 0.0;
        const int64_t i = min(i0 + r, M - 1);
        arow[r] = A + i * lda;
        klo[r] = tri == 1 ? i0 + r : 0;                   // rows past M: empty range
        khi[r] = i0 + r >= M ? 0 : tri == 2 ? min(K, i0 + r + 1) : K;
    }
    for (int64_t k = kb + lane; k < ke; k += 64) {
        double bv[MM];
#pragma unroll
        for (int c = 0; c < MM; ++c) bv[c] = c < m ? B[k * ldb + c] : 0.0;
#pragma unroll
        for (int r = 0; r < RP; ++r) {
            const double a = (k >= klo[r] && k < khi[r]) ? arow[r][k] : 0.0;
#pragma unroll
            for (int c = 0; c < MM; ++c) acc[r][c] += a * bv[c];
        }
    }
    // the RP MM sums by a halving exchange across the lanes: at offset o a
    // lane keeps half of its partial sums (the upper half when lane & o) and
    // adds its partner's values of that half, so each sum is formed by a
    // butterfly's pairwise tree; value r MM + c ends in lane (r MM + c) DUP
    constexpr int V = RP * MM;
    static_assert(V <= 64 && (V & (V - 1)) == 0, "a power-of-two count of sums");
    constexpr int DUP = 64 / V;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int o = 32 >> k, n = V >> k;
        if (n > 1) {
            const bool up = (lane & o) != 0;
#pragma unroll
            for (int q = 0; q < n / 2; ++q) {
                double& lo = acc[q / MM][q % MM];
                const double hi = acc[(q + n / 2) / MM][(q + n / 2) % MM];
                const double send = up ? lo : hi, keep = up ? hi : lo;
                lo = keep + __shfl_xor(send, o);
            }
        } else {
            acc[0][0] += __shfl_xor(acc[0][0], o);
        }
    }
    const int idx = lane / DUP, r = idx / MM, c = idx % MM;
    const int64_t i = i0 + r;
    if (lane % DUP == 0 && c < m && i < M) {
        double v = alpha * acc[0][0];
        if (beta != 0.0) v += beta * C[i * ldc + c];
        C[i * ldc + c] = v;
    }
}

template <int MM>
__global__ __launch_bounds__(256) void rowprod_kernel(int64_t M, int64_t K, int m, double alpha,
                                                      const double* __restrict__ A, int64_t lda,
                                                      int tri, const double* __restrict__ B,
                                                      int64_t ldb, double beta, double* C,
                                                      int64_t ldc) {
    rowprod_body<MM>(blockIdx.x, M, K, m, alpha, A, lda, tri, B, ldb, beta, C, ldc);
}

template <int MM>
__global__ __launch_bounds__(256) void rowprod_grouped(const RowprodDesc* __restrict__ d,
                                                       GroupSched g) {
    int64_t lb;
    const int j = group_problem(g, lb);
    if (!group_live(g, j)) return;
    const RowprodDesc& q = d[j];
    rowprod_body<MM>(lb, q.M, q.K, q.m, q.alpha, q.A, q.lda, q.tri, q.B, q.ldb, q.beta, q.C, q.ldc);
}

// row copies of the grouped apply, one element per thread
template <bool SCATTER>
__global__ __launch_bounds__(256) void copy_rows_grouped(const CopyRowsDesc* __restrict__ d,
                                                         GroupSched g) {
    int64_t lb;
    const int jp = group_problem(g, lb);
    if (!group_live(g, jp)) return;
    const CopyRowsDesc& q = d[jp];
    const int64_t e = lb * 256 + threadIdx.x;
    if (e >= q.rows * q.cols) return;
    const int64_t i = e / q.cols, c = e % q.cols;
    const int64_t j = q.idx[i];
    if (SCATTER)
        q.dst[j * q.ldd + c] = q.src[i * q.lds + c];
    else
        q.dst[i * q.ldd + c] = q.src[j * q.lds + c];
}

// B = A^T for an R x C matrix A (ld lda) into B (C x R, ld ldb)
__device__ __forceinline__ void transpose_body(int64_t bx, int64_t by, int64_t R, int64_t Cn,
                                               const double* __restrict__ A, int64_t lda,
                                               double* __restrict__ B, int64_t ldb) {
    __shared__ double t[32][33];
    const int64_t r0 = by * 32, c0 = bx * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + threadIdx.x;
        if (r < R && c < Cn) t[k][threadIdx.x] = A[r * lda + c];
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + threadIdx.x;
        if (r < R && c < Cn) B[c * ldb + r] = t[threadIdx.x][k];
    }
}

__global__ void transpose_kernel(int64_t R, int64_t Cn, const double* __restrict__ A, int64_t lda,
                                 double* __restrict__ B, int64_t ldb) {
    transpose_body(blockIdx.x, blockIdx.y, R, Cn, A, lda, B, ldb);
}

// the matrix steps of grouped factor tails (MatOp); element-wise steps take
// one element per thread, in blocks of 256
template <MatOp OP>
__global__ __launch_bounds__(256) void mat_grouped(const MatDesc* __restrict__ d, GroupSched g) {
    int64_t lb;
    const MatDesc& q = d[group_problem(g, lb)];
    if constexpr (OP == MatOp::TRANSPOSE) {
        const int64_t nbx = cdiv(q.cols, 32);
        transpose_body(lb % nbx, lb / nbx, q.rows, q.cols, q.src, q.lds, q.dst, q.ldd);
    } else if constexpr (OP == MatOp::TRTRI_LEAF) {
        trtri_leaf_body(lb, q.rows, q.src, q.lds, q.dst, q.ldd);
    } else if constexpr (OP == MatOp::ADD_IDENTITY) {
        const int64_t e = lb * 256 + threadIdx.x;
        if (e < q.rows) q.dst[e * q.ldd + e] += 1.0;
    } else {
        const int64_t e = lb * 256 + threadIdx.x;
        if (e >= q.rows * q.cols) return;
        const int64_t i = e / q.cols, j = e % q.cols;
        if constexpr (OP == MatOp::ZERO) q.dst[i * q.ldd + j] = 0.0;
        if constexpr (OP == MatOp::GATHER_COLS) q.dst[i * q.ldd + j] = q.src[i * q.lds + q.idx[j]];
    }
}

}  // namespace

void rowprod(hipStream_t s, int64_t M, int64_t K, int64_t m, double alpha, const double* A, int64_t lda,
             int tri, const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
    if (M <= 0) return;
    const int mi = (int)m;
#define ELM_RP(MM)                                                                                  \
    rowprod_kernel<MM><<<(unsigned)cdiv(M, Rowprod<MM>::RB), 256, 0, s>>>(M, K, mi, alpha, A, lda, tri, B, \
                                                                         ldb, beta, C, ldc)
    if (m <= 4)
        ELM_RP(4);
    else if (m <= 8)
        ELM_RP(8);
    else if (m <= 16)
        ELM_RP(16);
    else
        ELM_RP(64);
#undef ELM_RP
    ELM_LAUNCH_CHECK();
}

// B (Cn x R, ld R) = A^T; returns B
double* transposed_copy(hipStream_t s, int64_t R, int64_t Cn, const double* A, int64_t lda,
                        double* B) {
    transpose_kernel<<<dim3((unsigned)cdiv(Cn, 32), (unsigned)cdiv(R, 32)), dim3(32, 8), 0, s>>>(R, Cn, A,
                                                                                                lda, B, R);
    ELM_LAUNCH_CHECK();
    return B;
}

void gather_rows(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds,
                 const int32_t* idx, double* dst, int64_t ldd) {
    if (rows <= 0 || cols <= 0) return;
    gather_rows_kernel<<<dim3((unsigned)cdiv(cols, 256), (unsigned)rows), 256, 0, s>>>(
        rows, cols, src, lds, idx, dst, ldd);
    ELM_LAUNCH_CHECK();
}

void scatter_rows(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds,
                  const int32_t* idx, double* dst, int64_t ldd) {
    if (rows <= 0 || cols <= 0) return;
    scatter_rows_kernel<<<dim3((unsigned)cdiv(cols, 256), (unsigned)rows), 256, 0, s>>>(
        rows, cols, src, lds, idx, dst, ldd);
    ELM_LAUNCH_CHECK();
}

void zero_mat(hipStream_t s, int64_t rows, int64_t cols, double* A, int64_t lda) {
    if (rows <= 0 || cols <= 0) return;
    zero_mat_kernel<<<dim3((unsigned)cdiv(cols, 256), (unsigned)rows), 256, 0, s>>>(rows, cols, A,
                                                                                   lda);
    ELM_LAUNCH_CHECK();
}

// X = U^-1 for upper-triangular U (r x r); X must not alias U.
void trtri_upper(hipStream_t s, int64_t r, const double* U, int64_t ldu, double* X, int64_t ldx,
                 Workspace& ws) {
    zero_mat(s, r, r, X, ldx);
    trtri_leaf_kernel<<<(unsigned)cdiv(r, LB), LB, 0, s>>>(r, U, ldu, X, ldx);
    ELM_LAUNCH_CHECK();
    // level sz joins pairs of inverted diagonal blocks a = [a0, a0 + sz),
    // c = [a0 + sz, a0 + 2 sz):  X[a, c] = -X[a, a] U[a, c] X[c, c].
    // The full-size pairs of a level share one launch per product; a ragged
    // last pair gets its own.
    size_t t1_max = 0;
    for (int64_t sz = LB; sz < r; sz *= 2) {
        const int64_t full = r / (2 * sz);
        size_t need = (size_t)full * sz * sz;
        if (full * 2 * sz + sz < r) need += (size_t)sz * sz;
        if (need > t1_max) t1_max = need;
    }
    double* T1 = t1_max ? (double*)ws.get("trtri_T1", t1_max * sizeof(double)) : nullptr;
    for (int64_t sz = LB; sz < r; sz *= 2) {
        const int64_t full = r / (2 * sz);  // pairs with both halves of size sz
        const int64_t pstride_u = 2 * sz * (ldu + 1), pstride_x = 2 * sz * (ldx + 1);
        if (full > 0) {
            // T1_p = U[a, c] X[c, c]   (X[c, c] upper triangular)
            gemm_f64_batched(s, full, sz, sz, sz, 1.0, U + sz, ldu, 1, pstride_u, X + sz * ldx + sz, ldx,
                             1, pstride_x, 0.0, T1, sz, sz * sz, false, true);
            // X[a, c] = -X[a, a] T1_p   (X[a, a] upper triangular)
            gemm_f64_batched(s, full, sz, sz, sz, -1.0, X, ldx, 1, pstride_x, T1, sz, 1, sz * sz, 0.0,
                             X + sz, ldx, pstride_x, true, false);
        }
        const int64_t a0 = full * 2 * sz, c0 = a0 + sz;
        if (c0 < r) {
            const int64_t nc = r - c0;
            double* T1r = T1 + (size_t)full * sz * sz;
            gemm_f64_batched(s, 1, sz, nc, nc, 1.0, U + a0 * ldu + c0, ldu, 1, 0, X + c0 * ldx + c0, ldx,
                             1, 0, 0.0, T1r, nc, 0, false, true);
            gemm_f64_batched(s, 1, sz, nc, sz, -1.0, X + a0 * ldx + a0, ldx, 1, 0, T1r, nc, 1, 0, 0.0,
                             X + a0 * ldx + c0, ldx, 0, true, false);
        }
    }
}

namespace {

// Y (q x m, ld m) <- S^-1 Y with S^-1 = Usinv Usinv^T (S = Us^T Us)
void apply_s_inv(hipStream_t s, const elm_factor* f, int64_t m, double* Y, Workspace& ws) {
    const int64_t q = f->q;
    double* t = (double*)ws.get("ap_sinv", (size_t)q * m * sizeof(double));
    rowprod(s, q, q, m, 1.0, f->UsinvT, q, 2, Y, m, 0.0, t, m);     // t = Usinv^T Y
    rowprod(s, q, q, m, 1.0, f->Usinv, q, 1, t, m, 0.0, Y, m);      // Y = Usinv t
}

// u (r x m) <- (G G^T)^-1 u = (I + K K^T)^-1 u
void apply_g_gram_inv(hipStream_t s, const elm_factor* f, int64_t m, double* u, Workspace& ws) {
    const int64_t r = f->r, c = f->n - f->r;
    if (f->q == 0) return;
    if (f->woodbury) {
        // (I + K K^T)^-1 = I - K (I + K^T K)^-1 K^T
        double* w = (double*)ws.get("ap_w", (size_t)c * m * sizeof(double));
        rowprod(s, c, r, m, 1.0, f->KT, r, 0, u, m, 0.0, w, m);      // w = K^T u
        apply_s_inv(s, f, m, w, ws);                                 // w = S'^-1 w
        rowprod(s, r, c, m, -1.0, f->K, c, 0, w, m, 1.0, u, m);      // u -= K w
    } else {
        apply_s_inv(s, f, m, u, ws);
    }
}

// y (r x m) <- (F^T F)^-1 y = R11^-1 R11^-T y
void apply_f_gram_inv(hipStream_t s, const elm_factor* f, int64_t m, double* y, Workspace& ws) {
    const int64_t r = f->r;
    double* t = (double*)ws.get("ap_finv", (size_t)r * m * sizeof(double));
    rowprod(s, r, r, m, 1.0, f->RinvT, r, 2, y, m, 0.0, t, m);      // t = Rinv^T y
    rowprod(s, r, r, m, 1.0, f->Rinv, r, 1, t, m, 0.0, y, m);       // y = Rinv t
}

}  // namespace

int64_t mat_group_blocks(MatOp op, const MatDesc& q) {
    switch (op) {
        case MatOp::TRANSPOSE: return cdiv(q.cols, 32) * cdiv(q.rows, 32);
        case MatOp::TRTRI_LEAF: return cdiv(q.rows, LB);
        case MatOp::ADD_IDENTITY: return cdiv(q.rows, 256);
        case MatOp::CHOL_INV_SMALL: return q.rows > 0 ? 1 : 0;
        default: return cdiv(q.rows * q.cols, 256);
    }
}

void launch_mat_grouped(hipStream_t s, MatOp op, const MatDesc* d, const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    const unsigned grid = (unsigned)g.blocks;
    switch (op) {
        case MatOp::ZERO: mat_grouped<MatOp::ZERO><<<grid, 256, 0, s>>>(d, g); break;
        case MatOp::TRANSPOSE: mat_grouped<MatOp::TRANSPOSE><<<grid, dim3(32, 8), 0, s>>>(d, g); break;
        case MatOp::ADD_IDENTITY: mat_grouped<MatOp::ADD_IDENTITY><<<grid, 256, 0, s>>>(d, g); break;
        case MatOp::GATHER_COLS: mat_grouped<MatOp::GATHER_COLS><<<grid, 256, 0, s>>>(d, g); break;
        case MatOp::TRTRI_LEAF: mat_grouped<MatOp::TRTRI_LEAF><<<grid, LB, 0, s>>>(d, g); break;
        case MatOp::CHOL_INV_SMALL: launch_chol_inv_small_grouped(s, d, g); return;
    }
    ELM_LAUNCH_CHECK();
}

int64_t rowprod_group_blocks(const RowprodDesc& q, int maxm) {
    const int64_t rb = maxm <= 16 ? Rowprod<16>::RB : Rowprod<64>::RB;  // the launch's template
    return q.M > 0 ? cdiv(q.M, rb) : 0;
}

int64_t copy_rows_group_blocks(const CopyRowsDesc& q) { return cdiv(q.rows * q.cols, 256); }

void launch_rowprod_grouped(hipStream_t s, const RowprodDesc* d, const GroupSched& g, int maxm) {
    if (g.count <= 0 || g.blocks <= 0) return;
    const unsigned grid = (unsigned)g.blocks;
    // the template follows the single-problem rule; the products do not depend on it
    if (maxm <= 4)
        rowprod_grouped<4><<<grid, 256, 0, s>>>(d, g);
    else if (maxm <= 8)
        rowprod_grouped<8><<<grid, 256, 0, s>>>(d, g);
    else if (maxm <= 16)
        rowprod_grouped<16><<<grid, 256, 0, s>>>(d, g);
    else
        rowprod_grouped<64><<<grid, 256, 0, s>>>(d, g);
    ELM_LAUNCH_CHECK();
}

void launch_copy_rows_grouped(hipStream_t s, bool scatter, const CopyRowsDesc* d,
                              const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    if (scatter)
        copy_rows_grouped<true><<<(unsigned)g.blocks, 256, 0, s>>>(d, g);
    else
        copy_rows_grouped<false><<<(unsigned)g.blocks, 256, 0, s>>>(d, g);
    ELM_LAUNCH_CHECK();
}

void build_factor_tail(hipStream_t s, elm_factor* f, Workspace& ws, bool wait) {
    const int64_t r = f->r, n = f->n, c = n - r;
    if (r == 0) return;
    f->Rinv = (double*)factor_alloc(f, "Rinv", (size_t)r * r * sizeof(double));
    trtri_upper(s, r, f->R, n, f->Rinv, r, ws);
    f->RinvT = transposed_copy(s, r, r, f->Rinv, r,
                               (double*)factor_alloc(f, "RinvT", (size_t)r * r * sizeof(double)));
    if (c > 0) {
        f->K = (double*)factor_alloc(f, "K", (size_t)r * c * sizeof(double));
        // K = R11^-1 R12 (R11^-1 upper triangular)
        gemm_f64_batched(s, 1, r, c, r, 1.0, f->Rinv, r, 1, 0, f->R + r, n, 1, 0, 0.0, f->K, c, 0, true,
                         false);
        f->KT = transposed_copy(s, r, c, f->K, c,
                                (double*)factor_alloc(f, "KT", (size_t)r * c * sizeof(double)));
    }
    const int64_t q = r < c ? r : c;
    f->q = q;
    f->woodbury = (c < r);
    if (q == 0) return;
    double* S = (double*)ws.get("ft_S", (size_t)q * q * sizeof(double));
    if (f->woodbury)
        gemm_f64(s, c, c, r, 1.0, f->K, 1, c, f->K, c, 1, 0.0, S, c);   // K^T K
    else
        gemm_f64(s, r, r, c, 1.0, f->K, c, 1, f->K, 1, c, 0.0, S, r);   // K K^T
    add_identity_kernel<<<(unsigned)cdiv(q, 256), 256, 0, s>>>(q, S, q);
    ELM_LAUNCH_CHECK();
    int* flag = (int*)ws.get("ft_flag", sizeof(int));
    ELM_HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
    f->Usinv = (double*)factor_alloc(f, "Usinv", (size_t)q * q * sizeof(double));
    if (q <= 128) {  // factor and inverse in one workgroup
        cholesky_inverse_small(s, q, S, q, f->Usinv, q, flag);
    } else {
        cholesky_blocked(s, q, S, q, 0.0, flag, ws);
        trtri_upper(s, q, S, q, f->Usinv, q, ws);
    }
    f->UsinvT = transposed_copy(s, q, q, f->Usinv, q,
                                (double*)factor_alloc(f, "UsinvT", (size_t)q * q * sizeof(double)));
    if (!wait) {  // the first solve reads the flag with its own synchronisation
        f->pd_flag = flag;
        return;
    }
    int hflag = 0;
    ELM_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    if (hflag) throw Error{ELM_ERR_NOT_PSD, "Gram of G is not positive definite"};
}

namespace {

void add_mat(GroupProgram& prog, MatOp op, const std::vector<MatDesc>& d) {
    std::vector<int64_t> nb(d.size());
    for (size_t j = 0; j < d.size(); ++j) nb[j] = mat_group_blocks(op, d[j]);
    prog.add(d, nb, [op](hipStream_t s, const void* dev, const GroupSched& g) {
        launch_mat_grouped(s, op, (const MatDesc*)dev, g);
    });
}

// products in two launches by the single-product tile rule
void add_gemm(GroupProgram& prog, const std::vector<GemmDesc>& d) {
    for (int ts : {128, 64}) {
        std::vector<GemmDesc> sel;
        std::vector<int64_t> nb;
        for (const GemmDesc& g : d)
            if (gemm_tile(g) == ts) {
                sel.push_back(g);
                nb.push_back(gemm_group_blocks(g, ts));
            }
        prog.add(sel, nb, [ts](hipStream_t s, const void* dev, const GroupSched& g) {
            launch_gemm_grouped(s, ts, (const GemmDesc*)dev, g);
        });
    }
}

GemmDesc gemm_desc(int64_t batch, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                   int64_t a_rs, int64_t a_cs, int64_t a_bs, const double* B, int64_t b_rs,
                   int64_t b_cs, int64_t b_bs, double beta, double* C, int64_t ldc, int64_t c_bs,
                   bool tri_a, bool tri_b) {
    GemmDesc g;
    g.batch = batch;
    g.M = M;
    g.N = N;
    g.K = K;
    g.alpha = alpha;
    g.A = A;
    g.a_rs = a_rs;
    g.a_cs = a_cs;
    g.a_bs = a_bs;
    g.B = B;
    g.b_rs = b_rs;
    g.b_cs = b_cs;
    g.b_bs = b_bs;
    g.beta = beta;
    g.C = C;
    g.ldc = ldc;
    g.c_bs = c_bs;
    g.tri_a = tri_a ? 1 : 0;
    g.tri_b = tri_b ? 1 : 0;
    return g;
}

// doubles of trtri_upper's level scratch for order r
size_t trtri_scratch(int64_t r) {
    size_t t1_max = 0;
    for (int64_t sz = LB; sz < r; sz *= 2) {
        const int64_t full = r / (2 * sz);
        size_t need = (size_t)full * sz * sz;
        if (full * 2 * sz + sz < r) need += (size_t)sz * sz;
        if (need > t1_max) t1_max = need;
    }
    return t1_max;
}

// X = U^-1 for several upper-triangular U: trtri_upper's steps, each level's
// products of every order in shared launches (a level's ragged pair is
// independent of its full pairs, so they share the launches too)
struct TriJob {
    int64_t r;
    const double* U;
    int64_t ldu;
    double* X;
    int64_t ldx;
    double* T1;  // trtri_scratch(r) doubles
};
void trtri_grouped(GroupProgram& prog, const std::vector<TriJob>& jobs) {
    std::vector<MatDesc> z, leaf;
    int64_t rmax = 0;
    for (const TriJob& j : jobs) {
        MatDesc a;
        a.rows = j.r;
        a.cols = j.r;
        a.dst = j.X;
        a.ldd = j.ldx;
        z.push_back(a);
        MatDesc b;
        b.rows = j.r;
        b.src = j.U;
        b.lds = j.ldu;
        b.dst = j.X;
        b.ldd = j.ldx;
        leaf.push_back(b);
        rmax = std::max(rmax, j.r);
    }
    add_mat(prog, MatOp::ZERO, z);
    add_mat(prog, MatOp::TRTRI_LEAF, leaf);
    for (int64_t sz = LB; sz < rmax; sz *= 2) {
        std::vector<GemmDesc> pa, pb;
        for (const TriJob& j : jobs) {
            const int64_t r = j.r;
            if (sz >= r) continue;
            const int64_t full = r / (2 * sz);
            const int64_t pstride_u = 2 * sz * (j.ldu + 1), pstride_x = 2 * sz * (j.ldx + 1);
            if (full > 0) {
                pa.push_back(gemm_desc(full, sz, sz, sz, 1.0, j.U + sz, j.ldu, 1, pstride_u,
                                       j.X + sz * j.ldx + sz, j.ldx, 1, pstride_x, 0.0, j.T1, sz,
                                       sz * sz, false, true));
                pb.push_back(gemm_desc(full, sz, sz, sz, -1.0, j.X, j.ldx, 1, pstride_x, j.T1, sz, 1,
                                       sz * sz, 0.0, j.X + sz, j.ldx, pstride_x, true, false));
            }
            const int64_t a0 = full * 2 * sz, c0 = a0 + sz;
            if (c0 < r) {
                const int64_t nc = r - c0;
                double* T1r = j.T1 + (size_t)full * sz * sz;
                pa.push_back(gemm_desc(1, sz, nc, nc, 1.0, j.U + a0 * j.ldu + c0, j.ldu, 1, 0,
                                       j.X + c0 * j.ldx + c0, j.ldx, 1, 0, 0.0, T1r, nc, 0, false, true));
                pb.push_back(gemm_desc(1, sz, nc, sz, -1.0, j.X + a0 * j.ldx + a0, j.ldx, 1, 0, T1r, nc,
                                       1, 0, 0.0, j.X + a0 * j.ldx + c0, j.ldx, 0, true, false));
            }
        }
        add_gemm(prog, pa);
        add_gemm(prog, pb);
    }
}

MatDesc transpose_desc(int64_t R, int64_t Cn, const double* A, int64_t lda, double* B) {
    MatDesc d;
    d.rows = R;
    d.cols = Cn;
    d.src = A;
    d.lds = lda;
    d.dst = B;
    d.ldd = R;
    return d;
}

}  // namespace

std::vector<int> build_factor_tails_grouped(hipStream_t s, const std::vector<elm_factor*>& fs,
                                            const std::vector<const double*>& Rorig, Workspace& ws) {
    const size_t P = fs.size();
    std::vector<int> bad(P, 0);
    if (P == 0) return bad;
    auto al = GroupProgram::al;
    // scratch: the level products of both inverses, the Gram of G, and a flag each
    std::vector<size_t> o_t1(P), o_s(P), o_t1s(P), o_w(P);
    size_t off = 0;
    for (size_t p = 0; p < P; ++p) {
        const elm_factor* f = fs[p];
        const int64_t r = f->r, c = f->n - r, q = std::min(r, c);
        if (r < 1) throw Error{ELM_ERR_INVALID_ARG, "grouped factor tail needs rank >= 1"};
        o_t1[p] = off;
        off += al(std::max<size_t>(trtri_scratch(r), 1) * sizeof(double));
        o_s[p] = off;
        off += al(std::max<size_t>((size_t)(q * q), 1) * sizeof(double));
        o_t1s[p] = off;
        off += al(std::max<size_t>(q > 128 ? trtri_scratch(q) : 0, 1) * sizeof(double));
        // two-block Grams of G: the first block's inverse and its block row, transposed
        o_w[p] = off;
        off += al(std::max<size_t>(q > 128 && q <= 256 ? (size_t)(128 * 128 + (q - 128) * 128) : 0, 1) *
                  sizeof(double));
    }
    const size_t o_flags = off;
    off += al(P * sizeof(int));
    char* sc = (char*)ws.get("tl_scratch", off);
    int* flags = (int*)(sc + o_flags);

    GroupProgram prog;
    std::vector<MatDesc> gat, tr_r, tr_k, addi, small, tr_s, t2, small2, zl2;
    std::vector<GemmDesc> kk, ss, u12, strip2;
    std::vector<TriJob> tri_r, tri_s;
    for (size_t p = 0; p < P; ++p) {
        elm_factor* f = fs[p];
        const int64_t r = f->r, n = f->n, c = n - r;
        if (Rorig[p]) {  // R = the first r rows of Rorig, columns in pivot order
            MatDesc d;
            d.rows = r;
            d.cols = n;
            d.src = Rorig[p];
            d.lds = n;
            d.idx = f->piv;
            d.dst = f->R;
            d.ldd = n;
            gat.push_back(d);
        }
        f->Rinv = (double*)factor_alloc(f, "Rinv", (size_t)r * r * sizeof(double));
        f->RinvT = (double*)factor_alloc(f, "RinvT", (size_t)r * r * sizeof(double));
        tri_r.push_back(TriJob{r, f->R, n, f->Rinv, r, (double*)(sc + o_t1[p])});
        tr_r.push_back(transpose_desc(r, r, f->Rinv, r, f->RinvT));
        if (c > 0) {
            f->K = (double*)factor_alloc(f, "K", (size_t)r * c * sizeof(double));
            f->KT = (double*)factor_alloc(f, "KT", (size_t)r * c * sizeof(double));
            // K = R11^-1 R12 (R11^-1 upper triangular)
            kk.push_back(gemm_desc(1, r, c, r, 1.0, f->Rinv, r, 1, 0, f->R + r, n, 1, 0, 0.0, f->K, c, 0,
                                   true, false));
            tr_k.push_back(transpose_desc(r, c, f->K, c, f->KT));
        }
        const int64_t q = r < c ? r : c;
        f->q = q;
        f->woodbury = (c < r);
        if (q == 0) continue;
        double* S = (double*)(sc + o_s[p]);
        if (f->woodbury)  // K^T K
            ss.push_back(gemm_desc(1, c, c, r, 1.0, f->K, 1, c, 0, f->K, c, 1, 0, 0.0, S, c, 0, false, false));
        else  // K K^T
            ss.push_back(gemm_desc(1, r, r, c, 1.0, f->K, c, 1, 0, f->K, 1, c, 0, 0.0, S, r, 0, false, false));
        MatDesc a;
        a.rows = q;
        a.dst = S;
        a.ldd = q;
        addi.push_back(a);
        f->Usinv = (double*)factor_alloc(f, "Usinv", (size_t)q * q * sizeof(double));
        f->UsinvT = (double*)factor_alloc(f, "UsinvT", (size_t)q * q * sizeof(double));
        if (q <= 128) {  // factor and inverse in one workgroup
            MatDesc d;
            d.rows = q;
            d.dst = S;
            d.ldd = q;
            d.aux = f->Usinv;
            d.lda = q;
            d.flag = flags + p;
            small.push_back(d);
        } else {
            tri_s.push_back(TriJob{q, S, q, f->Usinv, q, (double*)(sc + o_t1s[p])});
            if (q <= 256) {
                // two diagonal blocks: the steps of the blocked factorisation
                // (first block, U12 = W^T T, the second block row's update,
                // second block), each shared by every such problem; every
                // element is computed as in the single-problem factorisation
                const int64_t q2 = q - 128;
                double* W = (double*)(sc + o_w[p]);
                double* Tt = W + 128 * 128;
                MatDesc d1;
                d1.rows = 128;
                d1.dst = S;
                d1.ldd = q;
                d1.aux = W;
                d1.lda = 128;
                d1.flag = flags + p;
                small.push_back(d1);
                t2.push_back(transpose_desc(128, q2, S + 128, q, Tt));
                u12.push_back(gemm_desc(1, 128, q2, 128, 1.0, W, 1, 128, 0, Tt, 1, 128, 0, 0.0, S + 128, q,
                                        0, false, false));
                strip2.push_back(gemm_desc(1, q2, q2, 128, -1.0, S + 128, 1, q, 0, S + 128, q, 1, 0, 1.0,
                                           S + 128 * q + 128, q, 0, false, false));
                MatDesc d2;
                d2.rows = q2;
                d2.dst = S + 128 * q + 128;
                d2.ldd = q;
                d2.aux = W;  // the first block's inverse is no longer needed
                d2.lda = 128;
                d2.flag = flags + p;
                small2.push_back(d2);
                MatDesc z;  // below the diagonal: zero, as the factorisation leaves it
                z.rows = q2;
                z.cols = 128;
                z.dst = S + 128 * q;
                z.ldd = q;
                zl2.push_back(z);
            }
        }
        tr_s.push_back(transpose_desc(q, q, f->Usinv, q, f->UsinvT));
    }
    add_mat(prog, MatOp::GATHER_COLS, gat);
    trtri_grouped(prog, tri_r);
    add_mat(prog, MatOp::TRANSPOSE, tr_r);
    add_gemm(prog, kk);
    add_mat(prog, MatOp::TRANSPOSE, tr_k);
    add_gemm(prog, ss);
    add_mat(prog, MatOp::ADD_IDENTITY, addi);
    add_mat(prog, MatOp::CHOL_INV_SMALL, small);
    add_mat(prog, MatOp::TRANSPOSE, t2);
    add_gemm(prog, u12);
    add_gemm(prog, strip2);
    add_mat(prog, MatOp::CHOL_INV_SMALL, small2);
    add_mat(prog, MatOp::ZERO, zl2);
    // larger Grams of G: the blocked factorisation one at a time, then the
    // inverses of all of them together
    for (size_t p = 0; p < P; ++p) {
        const int64_t q = fs[p]->q;
        if (q <= 256) continue;
        double* S = (double*)(sc + o_s[p]);
        int* flag = flags + p;
        prog.call([=, &ws] { cholesky_blocked(s, q, S, q, 0.0, flag, ws); });
    }
    trtri_grouped(prog, tri_s);
    add_mat(prog, MatOp::TRANSPOSE, tr_s);
    ELM_HIP_TRY(hipMemsetAsync(flags, 0, P * sizeof(int), s));
    prog.run(s, ws, "tl_program");
    std::vector<int> hf(P, 0);
    ELM_HIP_TRY(hipMemcpyAsync(hf.data(), flags, P * sizeof(int), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    ++ws.host_syncs;
    for (size_t p = 0; p < P; ++p) bad[p] = hf[p] ? 1 : 0;
    return bad;
}

// out (L x m) = H^+ (.) through the factor.
//   N >= L: rhs is H^T (.)  (L x m, ld ldr).
//   N <  L: rhs is (.) itself (N x m, ld ldr); H64 (N x L sample-major) supplies F'.
void apply_pinv(hipStream_t s, const elm_factor* f, int64_t m, const double* rhs, int64_t ldr,
                const double* H64, int64_t ldh64, double* out, int64_t ldo, Workspace& ws) {
    const int64_t r = f->r, n = f->n, c = n - r, L = f->L;
    if (r == 0) {
        zero_mat(s, L, m, out, ldo);
        return;
    }
    double* u = (double*)ws.get("ap_u", (size_t)r * m * sizeof(double));
    if (!f->transposed) {
        gather_rows(s, r, m, rhs, ldr, f->piv, u, m);     // F^T (.) = rows piv[:r] of H^T (.)
        apply_f_gram_inv(s, f, m, u, ws);                 // (F^T F)^-1
        apply_g_gram_inv(s, f, m, u, ws);                 // (G G^T)^-1
        // beta[piv] = [u; K^T u]  (eq. 7 block order)
        scatter_rows(s, r, m, u, m, f->piv, out, ldo);
        if (c > 0) {
            double* bd = (double*)ws.get("ap_bd", (size_t)c * m * sizeof(double));
            rowprod(s, c, r, m, 1.0, f->KT, r, 0, u, m, 0.0, bd, m);    // K^T u
            scatter_rows(s, c, m, bd, m, f->piv + r, out, ldo);
        }
        return;
    }
    // N < L: w = G' rhs = rhs[piv[:r]] + K rhs[piv[r:]]
    gather_rows(s, r, m, rhs, ldr, f->piv, u, m);
    if (c > 0) {
        double* t2 = (double*)ws.get("ap_t2", (size_t)c * m * sizeof(double));
        gather_rows(s, c, m, rhs, ldr, f->piv + r, t2, m);
        rowprod(s, r, c, m, 1.0, f->K, c, 0, t2, m, 1.0, u, m);        // u += K rhs[piv[r:]]
    }
    apply_g_gram_inv(s, f, m, u, ws);                     // (G' G'^T)^-1
    apply_f_gram_inv(s, f, m, u, ws);                     // (F'^T F')^-1
    double* G1 = (double*)ws.get("ap_G1", (size_t)r * L * sizeof(double));
    gather_rows(s, r, L, H64, ldh64, f->piv, G1, L);      // F'^T = H[piv[:r], :]
    gemm_f64(s, L, m, r, 1.0, G1, 1, L, u, m, 1, 0.0, out, ldo);
}

}  // namespace elm
