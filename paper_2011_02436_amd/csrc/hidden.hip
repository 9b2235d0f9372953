// Hidden layer of the ELM: H[i][j] = g(sum_k X[i][k] W[k][j] + b[j]), g the
// logistic sigmoid (Section 2.1, eqs. 1 and 4; step 2 of the RBP-ELM
// algorithm; Section 4 names the sigmoid).
//
// One fused kernel: an MFMA GEMM tile (16x16x4 FP64 or FP32 matrix
// instructions), bias add and sigmoid in registers, and up to two stores of
// the same values: the sample-major H (N x L, dtype of the inputs) used by the
// FP64 Gram and the refinement residual, and a node-major copy (L x N) rounded
// to nearest even in BF16/FP16/FP32 that feeds the low-precision Gram, whose
// MFMA operands want each hidden node's samples contiguous.
#include "elm_internal.h"

namespace elm {
namespace {

constexpr int BM = 64;   // samples per tile
constexpr int BN = 64;   // hidden nodes per tile
constexpr int BK = 16;   // reduction chunk over input features
constexpr int NT = 256;  // 4 waves, each a 32 x 32 sub-tile of 2 x 2 MFMA blocks

__device__ inline double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }
__device__ inline float sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

// Round-to-odd narrowing to float: keeps a sticky bit so that a second
// rounding to nearest even (to BF16/FP16) equals one direct rounding.
__device__ inline float narrow_odd(double x) {
    float f = __double2float_rz(x);
    if ((double)f != x) {
        uint32_t u = __float_as_uint(f) | 1u;
        f = __uint_as_float(u);
    }
    return f;
}
__device__ inline float narrow_odd(float x) { return x; }

__device__ inline uint16_t bf16_rne_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u)            // Inf/NaN: truncate, keep NaN quiet
        return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename T>
__device__ inline void store_lp(void* Hlp, elm_dtype lp, int64_t idx, T v) {
    if (lp == ELM_BF16) {
        ((uint16_t*)Hlp)[idx] = bf16_rne_bits(narrow_odd(v));
    } else if (lp == ELM_F16) {
        ((__half*)Hlp)[idx] = __float2half_rn(narrow_odd(v));
    } else {  // ELM_F32
        ((float*)Hlp)[idx] = (float)v;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void hidden_kernel(int64_t N, int64_t d, int64_t L,
                                                    const T* __restrict__ X, int64_t ldx,
                                                    const T* __restrict__ W, int64_t ldw,
                                                    const T* __restrict__ bias,
                                                    T* __restrict__ H, int64_t ldh,
                                                    void* __restrict__ Hlp, int64_t ldlp,
                                                    elm_dtype lp_dt) {
    __shared__ T Xs[BK][BM + 1];  // k-major so each MFMA A read is 16 consecutive samples
    __shared__ T Ws[BK][BN + 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t n0 = (int64_t)blockIdx.x * BM;
    const int64_t j0 = (int64_t)blockIdx.y * BN;

    typename Mfma16<T>::acc_t acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = typename Mfma16<T>::acc_t{};

    for (int64_t k0 = 0; k0 < d; k0 += BK) {
        // X tile: BM x BK, k fastest across threads (contiguous in X)
        for (int e = tid; e < BM * BK; e += NT) {
            int i = e / BK, k = e % BK;
            int64_t gi = n0 + i, gk = k0 + k;
            Xs[k][i] = (gi < N && gk < d) ? X[gi * ldx + gk] : T(0);
        }
        // W tile: BK x BN, j fastest (contiguous in W)
        for (int e = tid; e < BK * BN; e += NT) {
            int k = e / BN, j = e % BN;
            int64_t gk = k0 + k, gj = j0 + j;
            Ws[k][j] = (gk < d && gj < L) ? W[gk * ldw + gj] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int k = kk + (lane >> 4);
            T a0 = Xs[k][wm * 32 + (lane & 15)];
            T a1 = Xs[k][wm * 32 + 16 + (lane & 15)];
            T b0 = Ws[k][wn * 32 + (lane & 15)];
            T b1 = Ws[k][wn * 32 + 16 + (lane & 15)];
            acc[0][0] = Mfma16<T>::op(a0, b0, acc[0][0]);
            acc[0][1] = Mfma16<T>::op(a0, b1, acc[0][1]);
            acc[1][0] = Mfma16<T>::op(a1, b0, acc[1][0]);
            acc[1][1] = Mfma16<T>::op(a1, b1, acc[1][1]);
        }
        __syncthreads();
    }

    // epilogue: element (i, j) of each 16 x 16 block, see Mfma16<T>::row
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int64_t gj = j0 + wn * 32 + bj * 16 + (lane & 15);
        if (gj >= L) continue;
        const T bj_val = bias[gj];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = n0 + wm * 32 + bi * 16 + Mfma16<T>::row(lane, v);
                if (gi >= N) continue;
                const T h = sigmoid(acc[bi][bj][v] + bj_val);
                if (H) H[gi * ldh + gj] = h;
                if (Hlp) store_lp<T>(Hlp, lp_dt, gj * ldlp + gi, h);
            }
        }
    }
}

}  // namespace

void launch_hidden(hipStream_t s, elm_dtype dt, int64_t N, int64_t d, int64_t L, const void* X,
                   int64_t ldx, const void* W, int64_t ldw, const void* b, void* H, int64_t ldh,
                   void* Hlp, int64_t ldlp, elm_dtype lp_dt) {
    dim3 grid((unsigned)cdiv(N, BM), (unsigned)cdiv(L, BN));
    if (dt == ELM_F64) {
        hidden_kernel<double><<<grid, NT, 0, s>>>(N, d, L, (const double*)X, ldx, (const double*)W,
                                                  ldw, (const double*)b, (double*)H, ldh, Hlp,
                                                  ldlp, lp_dt);
    } else {
        hidden_kernel<float><<<grid, NT, 0, s>>>(N, d, L, (const float*)X, ldx, (const float*)W,
                                                 ldw, (const float*)b, (float*)H, ldh, Hlp, ldlp,
                                                 lp_dt);
    }
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
