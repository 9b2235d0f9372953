// General FP64 matrix product on the 16x16x4 FP64 MFMA, for the small dense
// steps after the rank reveal: K = R11^-1 R12, the Gram I + K K^T of G, the
// block triangular inverse and the applications of (F^T F)^-1 and
// (G G^T)^-1.  Operands are strided views, so transposes cost nothing:
//   C[i][j] = alpha * sum_k A(i, k) B(k, j) + beta * C[i][j],
//   A(i, k) = A[i * a_rs + k * a_cs],  B(k, j) = B[k * b_rs + j * b_cs].
#include "elm_internal.h"

namespace elm {
namespace {

constexpr int T = 64;   // output tile
constexpr int BK = 16;
constexpr int NT = 256;

__global__ __launch_bounds__(NT) void gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                  const double* __restrict__ A, int64_t a_rs,
                                                  int64_t a_cs, const double* __restrict__ B,
                                                  int64_t b_rs, int64_t b_cs, double beta,
                                                  double* __restrict__ C, int64_t ldc) {
    __shared__ double As[BK][T + 1];
    __shared__ double Bs[BK][T + 1];
    const int64_t i0 = (int64_t)blockIdx.x * T, j0 = (int64_t)blockIdx.y * T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const bool a_icontig = (a_rs == 1);
    const bool b_jcontig = (b_cs == 1);

    d4v acc[2][2];
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y) acc[x][y] = d4v{};

    for (int64_t k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int it = 0; it < (BK * T) / NT; ++it) {
            const int e = tid + it * NT;
            int i, k;
            if (a_icontig) { k = e / T; i = e % T; } else { i = e / BK; k = e % BK; }
            const int64_t gi = i0 + i, gk = k0 + k;
            As[k][i] = (gi < M && gk < K) ? A[gi * a_rs + gk * a_cs] : 0.0;
            int j, kb;
            if (b_jcontig) { kb = e / T; j = e % T; } else { j = e / BK; kb = e % BK; }
            const int64_t gj = j0 + j, gkb = k0 + kb;
            Bs[kb][j] = (gj < N && gkb < K) ? B[gkb * b_rs + gj * b_cs] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int k = kk + (lane >> 4);
            const double a0 = As[k][wm * 32 + (lane & 15)], a1 = As[k][wm * 32 + 16 + (lane & 15)];
            const double b0 = Bs[k][wn * 32 + (lane & 15)], b1 = Bs[k][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = Mfma16<double>::op(a0, b0, acc[0][0]);
            acc[0][1] = Mfma16<double>::op(a0, b1, acc[0][1]);
            acc[1][0] = Mfma16<double>::op(a1, b0, acc[1][0]);
            acc[1][1] = Mfma16<double>::op(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }
    for (int x = 0; x < 2; ++x)
        for (int y = 0; y < 2; ++y)
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = i0 + wm * 32 + x * 16 + Mfma16<double>::row(lane, v);
                const int64_t gj = j0 + wn * 32 + y * 16 + (lane & 15);
                if (gi >= M || gj >= N) continue;
                double c = alpha * acc[x][y][v];
                if (beta != 0.0) c += beta * C[gi * ldc + gj];
                C[gi * ldc + gj] = c;
            }
}

}  // namespace

void gemm_f64(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
              int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs, int64_t b_cs, double beta,
              double* C, int64_t ldc) {
    if (M <= 0 || N <= 0) return;
    dim3 grid((unsigned)cdiv(M, T), (unsigned)cdiv(N, T));
    gemm_kernel<<<grid, NT, 0, s>>>(M, N, K, alpha, A, a_rs, a_cs, B, b_rs, b_cs, beta, C, ldc);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
