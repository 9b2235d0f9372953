// The paper's own block form of the least-squares solve (Section 3, eqs. 13-23)
// for a hidden matrix of full column rank, evaluated from the blocks of the
// Gram M = H^T H and of Z = H^T T after a column split H P = [H1 H2]
// (H1: the first s columns in the order P, H2: the other L - s):
//   A  = H2^T H2                                   (eq. 20)
//   B  = A^-1 H2^T T                               (eq. 21)
//   D  = H1^T C H1,  C = I - H2 A^-1 H2^T          (eqs. 22-23)
//      = M11 - M12 A^-1 M21   (C, N x N, is never formed)
//   beta1 = D^-1 H1^T (T - H2 B) = D^-1 (Z1 - M12 B)   (eq. 19, first block;
//                                  the transpose on H1 is the one eq. 19 omits)
//   beta2 = B - A^-1 M21 beta1                     (eq. 19, second block)
//   beta[P] = [beta1; beta2]                       (eq. 7's block order)
// With A = Ua^T Ua and Xa = Ua^-1:  A^-1 = Xa Xa^T, V = Xa^T M21 and
// M12 A^-1 M21 = V^T V, so D comes from one product of V with itself, and
// A^-1 M21 beta1 = Xa (V beta1).  A pivot of A's or D's Cholesky at or below
// thr (the rank step's threshold) means a column that is numerically a
// combination of others: the block form then has no solution.  All FP64:
// the blocked (or one-workgroup) Cholesky and triangular inverse of the rank
// step, FP64 MFMA products, and the thin products of the solves.
#include "elm_internal.h"

#include <algorithm>

namespace elm {
namespace {

// dst[i][j] = M[p(r0 + i)][p(c0 + j)], p = piv or the identity
__global__ void gather_block_kernel(int64_t rows, int64_t cols, const double* __restrict__ M,
                                    int64_t ldm, const int32_t* __restrict__ piv, int64_t r0,
                                    int64_t c0, double* __restrict__ dst, int64_t ldd) {
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows || j >= cols) return;
    const int64_t gi = piv ? piv[r0 + i] : r0 + i;
    const int64_t gj = piv ? piv[c0 + j] : c0 + j;
    dst[i * ldd + j] = M[gi * ldm + gj];
}

void gather_block(hipStream_t s, int64_t rows, int64_t cols, const double* M, int64_t ldm,
                  const int32_t* piv, int64_t r0, int64_t c0, double* dst, int64_t ldd) {
    if (rows <= 0 || cols <= 0) return;
    gather_block_kernel<<<dim3((unsigned)cdiv(cols, 256), (unsigned)rows), 256, 0, s>>>(
        rows, cols, M, ldm, piv, r0, c0, dst, ldd);
    ELM_LAUNCH_CHECK();
}

__global__ void clear_int_kernel(int* p) {
    if (threadIdx.x == 0) p[0] = 0;
}

// A (q x q, ld q) = U^T U in place (upper triangle) and X = U^-1 (q x q, ld q);
// flag set at a pivot <= thr
void cholesky_and_inverse(hipStream_t s, int64_t q, double* A, double* X, int* flag, double thr,
                          Workspace& ws) {
    if (q <= 128) {
        cholesky_inverse_small(s, q, A, q, X, q, flag, thr);
    } else {
        cholesky_blocked(s, q, A, q, thr, flag, ws);
        trtri_upper(s, q, A, q, X, q, ws);
    }
}

}  // namespace

void block_solve(hipStream_t s, int64_t L, int64_t m, int64_t split, const double* M, int64_t ldm,
                 const double* Z, int64_t ldz, const int32_t* piv, double thr, double* beta, int64_t ldb,
                 Workspace& ws) {
    const int64_t s1 = split, s2 = L - split;
    int32_t* p = const_cast<int32_t*>(piv);
    if (!p) {  // the identity order, for the final scatter
        p = (int32_t*)ws.get("bs_iota", (size_t)L * sizeof(int32_t));
        launch_iota(s, L, p);
    }
    int* flag = (int*)ws.get("bs_flag", sizeof(int));
    clear_int_kernel<<<1, 64, 0, s>>>(flag);
    ELM_LAUNCH_CHECK();

    // D starts as M11; beta1's right-hand side as Z1
    double* D = (double*)ws.get("bs_D", (size_t)s1 * s1 * sizeof(double));
    double* XD = (double*)ws.get("bs_XD", (size_t)s1 * s1 * sizeof(double));
    double* rhs1 = (double*)ws.get("bs_rhs1", (size_t)s1 * m * sizeof(double));
    double* t1 = (double*)ws.get("bs_t1", (size_t)s1 * m * sizeof(double));
    gather_block(s, s1, s1, M, ldm, piv, 0, 0, D, s1);
    gather_rows(s, s1, m, Z, ldz, p, rhs1, m);

    double *M12 = nullptr, *XA = nullptr, *V = nullptr, *Bm = nullptr, *t2 = nullptr;
    if (s2 > 0) {
        double* A = (double*)ws.get("bs_A", (size_t)s2 * s2 * sizeof(double));
        XA = (double*)ws.get("bs_XA", (size_t)s2 * s2 * sizeof(double));
        double* XAT = (double*)ws.get("bs_XAT", (size_t)s2 * s2 * sizeof(double));
        M12 = (double*)ws.get("bs_M12", (size_t)s1 * s2 * sizeof(double));
        V = (double*)ws.get("bs_V", (size_t)s2 * s1 * sizeof(double));
        Bm = (double*)ws.get("bs_B", (size_t)s2 * m * sizeof(double));
        t2 = (double*)ws.get("bs_t2", (size_t)s2 * m * sizeof(double));
        gather_block(s, s2, s2, M, ldm, piv, s1, s1, A, s2);     // A = H2^T H2 (eq. 20)
        gather_block(s, s1, s2, M, ldm, piv, 0, s1, M12, s2);    // H1^T H2
        gather_rows(s, s2, m, Z, ldz, p + s1, t2, m);            // H2^T T
        cholesky_and_inverse(s, s2, A, XA, flag, thr, ws);       // A = Ua^T Ua, XA = Ua^-1
        transposed_copy(s, s2, s2, XA, s2, XAT);
        // B = XA XA^T H2^T T  (eq. 21)
        rowprod(s, s2, s2, m, 1.0, XAT, s2, 2, t2, m, 0.0, Bm, m);
        rowprod(s, s2, s2, m, 1.0, XA, s2, 1, Bm, m, 0.0, t2, m);
        std::swap(Bm, t2);
        // V = XA^T M21 (s2 x s1): A(i, k) = XA[k][i], B(k, j) = M12[j][k]
        gemm_f64(s, s2, s1, s2, 1.0, XA, 1, s2, M12, 1, s2, 0.0, V, s1);
        // D = M11 - V^T V = H1^T C H1  (eqs. 22-23)
        gemm_f64(s, s1, s1, s2, -1.0, V, 1, s1, V, s1, 1, 1.0, D, s1);
        // right-hand side of beta1: Z1 - M12 B = H1^T (T - H2 B)
        rowprod(s, s1, s2, m, -1.0, M12, s2, 0, Bm, m, 1.0, rhs1, m);
    }
    // beta1 = D^-1 rhs1 = XD XD^T rhs1  (eq. 19, first block)
    cholesky_and_inverse(s, s1, D, XD, flag, thr, ws);
    double* XDT = (double*)ws.get("bs_XDT", (size_t)s1 * s1 * sizeof(double));
    transposed_copy(s, s1, s1, XD, s1, XDT);
    rowprod(s, s1, s1, m, 1.0, XDT, s1, 2, rhs1, m, 0.0, t1, m);
    rowprod(s, s1, s1, m, 1.0, XD, s1, 1, t1, m, 0.0, rhs1, m);
    scatter_rows(s, s1, m, rhs1, m, p, beta, ldb);
    if (s2 > 0) {
        // beta2 = B - A^-1 M21 beta1 = B - XA (V beta1)  (eq. 19, second block)
        rowprod(s, s2, s1, m, 1.0, V, s1, 0, rhs1, m, 0.0, t2, m);
        rowprod(s, s2, s2, m, -1.0, XA, s2, 1, t2, m, 1.0, Bm, m);
        scatter_rows(s, s2, m, Bm, m, p + s1, beta, ldb);
    }
    int hflag = 0;
    ELM_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    if (hflag)
        throw Error{ELM_ERR_NOT_PSD, "a pivot of A = H2^T H2 or of D = H1^T C H1 is at or below the rank "
                                     "threshold: H is not of full column rank"};
}

}  // namespace elm
