// Prediction, step 3 of the three-step ELM (Section 2.1): Y = H beta with
// H = sigmoid(X W + b) recomputed tile by tile and never stored, and the
// arg-max label of each row (lowest index on ties; the training accuracy of
// Table 2 compares it with the class).
//
// One block owns 64 samples: for each tile of 64 hidden nodes it forms the
// 64 x 64 hidden tile on the 16x16x4 MFMA, applies bias and sigmoid, and
// accumulates the tile's product with the matching 64 rows of beta.
#include "elm_internal.h"

#include <cmath>

namespace elm {
namespace {

constexpr int RB = 64;   // samples per block
constexpr int NB = 64;   // hidden nodes per tile
constexpr int BK = 16;
constexpr int NT = 256;

__device__ inline double sigm(double z) { return 1.0 / (1.0 + exp(-z)); }
__device__ inline float sigm(float z) { return 1.0f / (1.0f + expf(-z)); }

template <typename T, int OPT>
__global__ __launch_bounds__(NT) void predict_kernel(int64_t N, int64_t d, int64_t L, int m,
                                                     const T* __restrict__ X, int64_t ldx,
                                                     const T* __restrict__ W, int64_t ldw,
                                                     const T* __restrict__ bias,
                                                     const double* __restrict__ beta, int64_t ldb,
                                                     T* __restrict__ Y, int64_t ldy,
                                                     int32_t* __restrict__ labels) {
    __shared__ T Xs[BK][RB + 1];
    __shared__ T Ws[BK][NB + 1];
    __shared__ T Hs[RB][NB + 1];
    __shared__ T Bs[NB][4 * OPT];
    __shared__ T Ys[RB][4 * OPT];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int row = tid & 63, grp = tid >> 6;
    const int64_t n0 = (int64_t)blockIdx.x * RB;

    T ya[OPT];
#pragma unroll
    for (int j = 0; j < OPT; ++j) ya[j] = T(0);

    for (int64_t j0 = 0; j0 < L; j0 += NB) {
        typename Mfma16<T>::acc_t acc[2][2];
        for (int a = 0; a < 2; ++a)
            for (int c = 0; c < 2; ++c) acc[a][c] = typename Mfma16<T>::acc_t{};
        for (int64_t k0 = 0; k0 < d; k0 += BK) {
            for (int e = tid; e < RB * BK; e += NT) {
                const int i = e / BK, k = e % BK;
                const int64_t gi = n0 + i, gk = k0 + k;
                Xs[k][i] = (gi < N && gk < d) ? X[gi * ldx + gk] : T(0);
            }
            for (int e = tid; e < BK * NB; e += NT) {
                const int k = e / NB, j = e % NB;
                const int64_t gk = k0 + k, gj = j0 + j;
                Ws[k][j] = (gk < d && gj < L) ? W[gk * ldw + gj] : T(0);
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int k = kk + (lane >> 4);
                const T a0 = Xs[k][wm * 32 + (lane & 15)], a1 = Xs[k][wm * 32 + 16 + (lane & 15)];
                const T b0 = Ws[k][wn * 32 + (lane & 15)], b1 = Ws[k][wn * 32 + 16 + (lane & 15)];
                acc[0][0] = Mfma16<T>::op(a0, b0, acc[0][0]);
                acc[0][1] = Mfma16<T>::op(a0, b1, acc[0][1]);
                acc[1][0] = Mfma16<T>::op(a1, b0, acc[1][0]);
                acc[1][1] = Mfma16<T>::op(a1, b1, acc[1][1]);
            }
            __syncthreads();
        }
        for (int bi = 0; bi < 2; ++bi)
            for (int bj = 0; bj < 2; ++bj)
                for (int v = 0; v < 4; ++v) {
                    const int i = wm * 32 + bi * 16 + Mfma16<T>::row(lane, v);
                    const int j = wn * 32 + bj * 16 + (lane & 15);
                    const int64_t gj = j0 + j;
                    Hs[i][j] = (gj < L) ? sigm(acc[bi][bj][v] + bias[gj]) : T(0);
                }
        for (int e = tid; e < NB * 4 * OPT; e += NT) {
            const int j = e / (4 * OPT), o = e % (4 * OPT);
            const int64_t gj = j0 + j;
            Bs[j][o] = (gj < L && o < m) ? (T)beta[gj * ldb + o] : T(0);
        }
        __syncthreads();
        for (int j = 0; j < NB; ++j) {
            const T h = Hs[row][j];
#pragma unroll
            for (int q = 0; q < OPT; ++q) ya[q] += h * Bs[j][grp + 4 * q];
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < OPT; ++q) Ys[row][grp + 4 * q] = ya[q];
    __syncthreads();
    const int64_t gi = n0 + row;
    if (gi < N) {
        if (Y)
            for (int q = 0; q < OPT; ++q) {
                const int o = grp + 4 * q;
                if (o < m) Y[gi * ldy + o] = ya[q];
            }
        if (labels && grp == 0) {
            int best = 0;
            T bv = Ys[row][0];
            for (int o = 1; o < m; ++o)
                if (Ys[row][o] > bv) { bv = Ys[row][o]; best = o; }
            labels[gi] = best;
        }
    }
}

template <typename T>
void run_predict(hipStream_t s, int64_t N, int64_t d, int64_t L, int64_t m, const T* X, int64_t ldx,
                 const T* W, int64_t ldw, const T* b, const double* beta, int64_t ldb, T* Y,
                 int64_t ldy, int32_t* labels) {
    const unsigned grid = (unsigned)cdiv(N, RB);
    const int mi = (int)m;
    if (m <= 4)
        predict_kernel<T, 1><<<grid, NT, 0, s>>>(N, d, L, mi, X, ldx, W, ldw, b, beta, ldb, Y, ldy, labels);
    else if (m <= 8)
        predict_kernel<T, 2><<<grid, NT, 0, s>>>(N, d, L, mi, X, ldx, W, ldw, b, beta, ldb, Y, ldy, labels);
    else if (m <= 16)
        predict_kernel<T, 4><<<grid, NT, 0, s>>>(N, d, L, mi, X, ldx, W, ldw, b, beta, ldb, Y, ldy, labels);
    else
        predict_kernel<T, 16><<<grid, NT, 0, s>>>(N, d, L, mi, X, ldx, W, ldw, b, beta, ldb, Y, ldy, labels);
    ELM_LAUNCH_CHECK();
}

}  // namespace

void launch_predict(hipStream_t s, elm_dtype dt, int64_t N, int64_t d, int64_t L, int64_t m,
                    const void* X, int64_t ldx, const void* W, int64_t ldw, const void* b,
                    const double* beta, int64_t ldbeta, void* Y, int64_t ldy, int32_t* labels,
                    Workspace&) {
    if (dt == ELM_F64)
        run_predict<double>(s, N, d, L, m, (const double*)X, ldx, (const double*)W, ldw,
                            (const double*)b, beta, ldbeta, (double*)Y, ldy, labels);
    else
        run_predict<float>(s, N, d, L, m, (const float*)X, ldx, (const float*)W, ldw,
                           (const float*)b, beta, ldbeta, (float*)Y, ldy, labels);
}

}  // namespace elm
