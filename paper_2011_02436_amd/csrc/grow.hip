// Incremental growth of the rank factor by new hidden nodes (a hidden-size
// sweep that reuses the work done for the smaller layer).
//
// The factor of H (N x n, Gram M = H^T H) holds the greedy pivoted Cholesky
// P^T M P = R^T R restricted to its r accepted positions: R = [R11 R12] (r x n
// in pivot order), R11^-1, and the rejected positions piv[r:].  Appending
// columns Hn (N x dn) gives H' = [H Hn] with the Gram
//   M' = [[M, C], [C^T, Gn]],  C = H^T Hn,  Gn = Hn^T Hn,
// of which only C and Gn are new (2 N n dn + N dn^2 flops instead of N n'^2).
// Keeping the r accepted pivots first, the rows of R extend over the new
// columns by X = R11^-T C[piv[:r], :], and the Schur complement of the first
// r positions restricted to the new columns is S = Gn - X^T X.  The greedy
// rule then continues on S: the old rejected positions never become pivots,
// because their Schur diagonals were already at most the old threshold (<=
// the new one, which grows with the order) and further pivots only lower
// them.  S's pivoted Cholesky gives the new pivots' rows over the new
// columns, R2 (r2 x dn); their entries over the old rejected positions solve
// R2_11^T Y = S_nr[piv2[:r2], :] with S_nr = C[piv[r:], :]^T - X^T R12.  The
// grown factor has rank r + r2, pivot order
//   [piv[:r], n + piv2[:r2], piv[r:], n + piv2[r2:]],
// R' = [[R11, X_acc, R12, X_rej], [0, R2_11, Y, R2_12]] in that order, and its
// tail (R11'^-1, K', the Gram of G) is formed as for any factor.  When the
// old decision would not stand under the grown threshold (an accepted pivot
// at or below it, or a rejected Schur diagonal above it) nothing is grown and
// the caller factors M' from scratch.  The rank and
// beta = H'^+ T are those of a factorisation of M' from scratch; the pivot
// order may differ (only r and beta are unique).
#include "elm_internal.h"

#include <algorithm>
#include <cmath>

namespace elm {
namespace {

// dst (rows x cols, ld ldd) += src^T for src (cols x rows, ld lds)
__global__ void add_transpose_kernel(int64_t rows, int64_t cols, const double* __restrict__ src,
                                     int64_t lds, double* __restrict__ dst, int64_t ldd) {
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows || j >= cols) return;
    dst[i * ldd + j] += src[j * lds + i];
}

// A (n x n, ld lda): the lower triangle takes the upper one's values, so the
// matrix is exactly symmetric
__global__ void mirror_upper_kernel(int64_t n, double* __restrict__ A, int64_t lda) {
    const int64_t i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || j >= i) return;
    A[i * lda + j] = A[j * lda + i];
}

// Rorig (rows x ncols, ld ldo) columns by original index: Rorig[i][map[p]] = src[i][p]
// for p < cols (src ld lds)
__global__ void scatter_cols_kernel(int64_t rows, int64_t cols, const double* __restrict__ src,
                                    int64_t lds, const int32_t* __restrict__ map, int32_t offset,
                                    double* __restrict__ Rorig, int64_t ldo) {
    const int64_t i = blockIdx.y;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows || p >= cols) return;
    const int64_t c = map ? (int64_t)map[p] + offset : p + offset;
    Rorig[i * ldo + c] = src[i * lds + p];
}

// the grown pivot order
__global__ void grown_piv_kernel(int64_t n, int64_t r, int64_t dn, int64_t r2, const int32_t* __restrict__ piv,
                                 const int32_t* __restrict__ piv2, int32_t* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n + dn) return;
    int32_t v;
    if (k < r) v = piv[k];
    else if (k < r + r2) v = (int32_t)n + piv2[k - r];
    else if (k < n + r2) v = piv[r + (k - r - r2)];
    else v = (int32_t)n + piv2[r2 + (k - n - r2)];
    out[k] = v;
}

void scatter_cols(hipStream_t s, int64_t rows, int64_t cols, const double* src, int64_t lds,
                  const int32_t* map, int32_t offset, double* Rorig, int64_t ldo) {
    if (rows <= 0 || cols <= 0) return;
    scatter_cols_kernel<<<dim3((unsigned)cdiv(cols, 256), (unsigned)rows), 256, 0, s>>>(
        rows, cols, src, lds, map, offset, Rorig, ldo);
    ELM_LAUNCH_CHECK();
}

}  // namespace

bool grow_factor(hipStream_t s, const elm_factor* f, int64_t N, int64_t L2, const double* H, int64_t ldh,
                 double tau_rel, elm_factor* g, Workspace& ws) {
    const int64_t n = f->n, r = f->r, c = n - r, dn = L2 - n, n2 = L2;
    // C' = H'^T Hn  (n2 x dn): rows [0, n) are C = H^T Hn, rows [n, n2) Gn
    double* Cf = (double*)ws.get("gr_C", (size_t)n2 * dn * sizeof(double));
    gemm_f64(s, n2, dn, N, 1.0, H, 1, ldh, H + n, ldh, 1, 0.0, Cf, dn);
    double* Gn = Cf + n * dn;
    // the largest diagonal of M' and the threshold (the default of
    // elm_rank_factor for the grown order)
    double* dmax = (double*)ws.get("gr_dmax", sizeof(double));
    launch_diag_max(s, dn, Gn, dn, dmax);
    double hmax = 0.0;
    ELM_HIP_TRY(hipMemcpyAsync(&hmax, dmax, sizeof(double), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    if (!std::isfinite(hmax)) throw Error{ELM_ERR_NOT_PSD, "Gram has a non-finite diagonal entry"};
    const double mx = std::max(f->max_diag, hmax);
    g->N = N;
    g->L = L2;
    g->n = n2;
    g->transposed = false;
    g->gram_dtype = ELM_F64;
    g->max_diag = mx;
    g->tau = (tau_rel > 0 ? tau_rel : 16.0 * (double)(n2 + N) * std::ldexp(1.0, -53)) * mx;
    g->noise_floor = schur_noise_floor(ELM_F64, n2, N, 0) * mx;
    g->device = f->device;
    // the old decision must stand under the grown threshold: every accepted
    // pivot above it, every rejected Schur diagonal at or below it
    if ((r > 0 && !(f->last_pivot > g->tau)) || (c > 0 && f->first_rejected > g->tau)) return false;

    // X = R11^-T C[piv[:r], :]  (r x dn)
    double* X = nullptr;
    if (r > 0) {
        double* C1 = (double*)ws.get("gr_C1", (size_t)r * dn * sizeof(double));
        X = (double*)ws.get("gr_X", (size_t)r * dn * sizeof(double));
        gather_rows(s, r, dn, Cf, dn, f->piv, C1, dn);
        gemm_f64(s, r, dn, r, 1.0, f->Rinv, 1, r, C1, dn, 1, 0.0, X, dn);   // A(i, k) = Rinv[k][i]
    }
    // S = Gn - X^T X, exactly symmetric
    double* S = (double*)ws.get("gr_S", (size_t)dn * dn * sizeof(double));
    ELM_HIP_TRY(hipMemcpy2DAsync(S, (size_t)dn * sizeof(double), Gn, (size_t)dn * sizeof(double),
                                 (size_t)dn * sizeof(double), (size_t)dn, hipMemcpyDeviceToDevice, s));
    if (r > 0) gemm_f64(s, dn, dn, r, -1.0, X, 1, dn, X, dn, 1, 1.0, S, dn);
    mirror_upper_kernel<<<dim3((unsigned)cdiv(dn, 256), (unsigned)dn), 256, 0, s>>>(dn, S, dn);
    ELM_LAUNCH_CHECK();

    // the greedy rule on S (its R2 and pivots in workspace buffers)
    elm_factor tmp;
    tmp.pool = &ws;
    int32_t* piv2 = (int32_t*)ws.get("gr_piv2", (size_t)dn * sizeof(int32_t));
    double* R2 = nullptr;
    double pst[3];
    const int64_t r2 = pivoted_cholesky(s, dn, S, dn, g->tau, piv2, &R2, pst, ws, &tmp);
    const int64_t r_new = r + r2;
    g->r = r_new;
    g->last_pivot = std::min(r > 0 ? f->last_pivot : INFINITY, pst[0]);
    // the old rejected positions' Schur diagonals only fell since the old stop
    g->first_rejected = std::max(c > 0 ? f->first_rejected : -INFINITY, pst[1]);
    g->reliable = (r_new == 0 || g->last_pivot >= 2.0 * g->noise_floor) &&
                  (r_new == n2 || g->first_rejected >= -2.0 * g->noise_floor);

    // the grown order and R' by original column index, then gathered
    g->piv = (int32_t*)factor_alloc(g, "piv", (size_t)n2 * sizeof(int32_t));
    grown_piv_kernel<<<(unsigned)cdiv(n2, 256), 256, 0, s>>>(n, r, dn, r2, f->piv, piv2, g->piv);
    ELM_LAUNCH_CHECK();
    if (r_new == 0) {
        g->R = nullptr;
        build_factor_tail(s, g, ws);
        return true;
    }
    double* Rorig = (double*)ws.get("gr_Rorig", (size_t)r_new * n2 * sizeof(double));
    zero_mat(s, r_new, n2, Rorig, n2);
    if (r > 0) {
        scatter_cols(s, r, n, f->R, n, f->piv, 0, Rorig, n2);      // old rows, old columns
        scatter_cols(s, r, dn, X, dn, nullptr, (int32_t)n, Rorig, n2);  // old rows, new columns
    }
    if (r2 > 0) {
        double* Rn = Rorig + r * n2;
        // new rows over the new columns: R2 is in S's pivot order
        scatter_cols(s, r2, dn, R2, dn, piv2, (int32_t)n, Rn, n2);
        if (c > 0) {
            // S_nr = C[piv[r:], :]^T - X^T R12  (dn x c), then its rows piv2[:r2]
            double* Snr = (double*)ws.get("gr_Snr", (size_t)dn * c * sizeof(double));
            zero_mat(s, dn, c, Snr, c);
            double* Crej = (double*)ws.get("gr_Crej", (size_t)c * dn * sizeof(double));
            gather_rows(s, c, dn, Cf, dn, f->piv + r, Crej, dn);
            add_transpose_kernel<<<dim3((unsigned)cdiv(c, 256), (unsigned)dn), 256, 0, s>>>(dn, c, Crej, dn,
                                                                                          Snr, c);
            ELM_LAUNCH_CHECK();
            if (r > 0) gemm_f64(s, dn, c, r, -1.0, X, 1, dn, f->R + r, n, 1, 1.0, Snr, c);
            double* Sp = (double*)ws.get("gr_Sp", (size_t)r2 * c * sizeof(double));
            gather_rows(s, r2, c, Snr, c, piv2, Sp, c);
            // Y = R2_11^-T Sp, R2_11 = the first r2 columns of R2 (upper triangular)
            double* R11b = (double*)ws.get("gr_R11b", (size_t)r2 * r2 * sizeof(double));
            double* Yi = (double*)ws.get("gr_Yi", (size_t)r2 * r2 * sizeof(double));
            double* Y = (double*)ws.get("gr_Y", (size_t)r2 * c * sizeof(double));
            ELM_HIP_TRY(hipMemcpy2DAsync(R11b, (size_t)r2 * sizeof(double), R2, (size_t)dn * sizeof(double),
                                         (size_t)r2 * sizeof(double), (size_t)r2, hipMemcpyDeviceToDevice,
                                         s));
            trtri_upper(s, r2, R11b, r2, Yi, r2, ws);
            gemm_f64(s, r2, c, r2, 1.0, Yi, 1, r2, Sp, c, 1, 0.0, Y, c);   // A(i, k) = Yi[k][i]
            scatter_cols(s, r2, c, Y, c, f->piv + r, 0, Rn, n2);
        }
    }
    g->R = (double*)factor_alloc(g, "R", (size_t)r_new * n2 * sizeof(double));
    launch_gather_rows(s, r_new, n2, Rorig, n2, g->piv, g->R, n2);
    build_factor_tail(s, g, ws);
    return true;
}

}  // namespace elm
