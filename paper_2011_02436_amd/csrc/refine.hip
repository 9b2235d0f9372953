// FP64 streaming passes over the sample-major FP64 hidden matrix H (N x L)
// for the normal-equation residual of beta = H^+ T (eqs. 5 and 8):
//   E = T - H beta           residual_kernel  (one pass over H)
//   G = H^T E, ||G||_F^2      ht_kernel + ht_reduce_kernel (one pass over H)
// G with E = T is the right-hand side H^T T of eq. (8).  Every sum runs in a
// fixed order (no atomics), so repeated runs are bitwise identical.
#include "elm_internal.h"

namespace elm {
namespace {

constexpr int RT = 64;     // rows per tile
constexpr int CT = 64;     // columns per tile
constexpr int NT = 256;
constexpr int HT_ROWS = 4096;  // rows per partial of H^T E

// OPT = outputs per thread = ceil(m / 4); thread t owns row t % 64 and the
// output columns c = t / 64 + 4 j.
template <int OPT>
__global__ __launch_bounds__(NT) void residual_kernel(int64_t N, int64_t L, int m,
                                                      const double* __restrict__ H, int64_t ldh,
                                                      const double* __restrict__ T, int64_t ldt,
                                                      const double* __restrict__ beta, int64_t ldb,
                                                      double* __restrict__ E, int64_t lde) {
    __shared__ double Hs[RT][CT + 1];
    __shared__ double Bs[CT][4 * OPT];
    const int tid = threadIdx.x;
    const int row = tid & 63, grp = tid >> 6;
    const int64_t n0 = (int64_t)blockIdx.x * RT;
    double acc[OPT];
#pragma unroll
    for (int j = 0; j < OPT; ++j) acc[j] = 0.0;

    for (int64_t c0 = 0; c0 < L; c0 += CT) {
        for (int e = tid; e < RT * CT; e += NT) {
            const int i = e / CT, c = e % CT;
            const int64_t gi = n0 + i, gc = c0 + c;
            Hs[i][c] = (gi < N && gc < L) ? H[gi * ldh + gc] : 0.0;
        }
        for (int e = tid; e < CT * 4 * OPT; e += NT) {
            const int c = e / (4 * OPT), o = e % (4 * OPT);
            const int64_t gc = c0 + c;
            Bs[c][o] = (gc < L && o < m) ? beta[gc * ldb + o] : 0.0;
        }
        __syncthreads();
        for (int c = 0; c < CT; ++c) {
            const double h = Hs[row][c];
#pragma unroll
            for (int j = 0; j < OPT; ++j) acc[j] += h * Bs[c][grp + 4 * j];
        }
        __syncthreads();
    }
    const int64_t gi = n0 + row;
    if (gi < N) {
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int o = grp + 4 * j;
            if (o < m) E[gi * lde + o] = (T ? T[gi * ldt + o] : 0.0) - acc[j];
        }
    }
}

// partial[chunk][col][o] = sum over the chunk's rows of H[row][col] E[row][o];
// thread t owns column t % 64 and outputs o = t / 64 + 4 j.
template <int OPT>
__global__ __launch_bounds__(NT) void ht_kernel(int64_t N, int64_t L, int m,
                                                const double* __restrict__ H, int64_t ldh,
                                                const double* __restrict__ E, int64_t lde,
                                                double* __restrict__ part) {
    __shared__ double Hs[RT][CT + 1];
    __shared__ double Es[RT][4 * OPT];
    const int tid = threadIdx.x;
    const int col = tid & 63, grp = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * CT;
    const int64_t rbeg = (int64_t)blockIdx.y * HT_ROWS;
    const int64_t rend = min(N, rbeg + HT_ROWS);
    double acc[OPT];
#pragma unroll
    for (int j = 0; j < OPT; ++j) acc[j] = 0.0;

    for (int64_t r0 = rbeg; r0 < rend; r0 += RT) {
        for (int e = tid; e < RT * CT; e += NT) {
            const int i = e / CT, c = e % CT;
            const int64_t gi = r0 + i, gc = c0 + c;
            Hs[i][c] = (gi < rend && gc < L) ? H[gi * ldh + gc] : 0.0;
        }
        for (int e = tid; e < RT * 4 * OPT; e += NT) {
            const int i = e / (4 * OPT), o = e % (4 * OPT);
            const int64_t gi = r0 + i;
            Es[i][o] = (gi < rend && o < m) ? E[gi * lde + o] : 0.0;
        }
        __syncthreads();
        for (int i = 0; i < RT; ++i) {
            const double h = Hs[i][col];
#pragma unroll
            for (int j = 0; j < OPT; ++j) acc[j] += h * Es[i][grp + 4 * j];
        }
        __syncthreads();
    }
    const int64_t gc = c0 + col;
    if (gc < L) {
        double* out = part + (int64_t)blockIdx.y * L * m;
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int o = grp + 4 * j;
            if (o < m) out[gc * m + o] = acc[j];
        }
    }
}

// G[i][o] = sum over chunks of the partials; per-block sum of squares
__global__ __launch_bounds__(NT) void ht_reduce_kernel(int64_t L, int m, int nchunk,
                                                       const double* __restrict__ part,
                                                       double* __restrict__ G, int64_t ldg,
                                                       double* __restrict__ sq_part) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    double sq = 0.0;
    if (e < L * m) {
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * L * m + e];
        G[(e / m) * ldg + (e % m)] = s;
        sq = s * s;
    }
    // fixed-shape tree over the block
    __shared__ double red[NT];
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sq_part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(NT) void sum_kernel(int64_t n, const double* __restrict__ x,
                                                 double* __restrict__ out) {
    __shared__ double red[NT];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NT) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void axpy_mat_kernel(int64_t rows, int64_t cols, const double* __restrict__ X,
                                int64_t ldx, double* __restrict__ Y, int64_t ldy) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < rows * cols) {
        const int64_t i = e / cols, j = e % cols;
        Y[i * ldy + j] += X[i * ldx + j];
    }
}

}  // namespace

void launch_residual(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H, int64_t ldh,
                     const double* T, int64_t ldt, const double* beta, int64_t ldb, double* E,
                     int64_t lde) {
    const unsigned grid = (unsigned)cdiv(N, RT);
    const int mi = (int)m;
    if (m <= 4)
        residual_kernel<1><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, T, ldt, beta, ldb, E, lde);
    else if (m <= 8)
        residual_kernel<2><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, T, ldt, beta, ldb, E, lde);
    else if (m <= 16)
        residual_kernel<4><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, T, ldt, beta, ldb, E, lde);
    else
        residual_kernel<16><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, T, ldt, beta, ldb, E, lde);
    ELM_LAUNCH_CHECK();
}

void launch_ht_times(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H, int64_t ldh,
                     const double* E, int64_t lde, double* G, int64_t ldg, double* nrm2,
                     Workspace& ws) {
    const int nchunk = (int)cdiv(N, HT_ROWS);
    double* part = (double*)ws.get("ht_part", (size_t)nchunk * L * m * sizeof(double));
    const unsigned nred = (unsigned)cdiv(L * m, NT);
    double* sq = (double*)ws.get("ht_sq", (size_t)nred * sizeof(double));
    dim3 grid((unsigned)cdiv(L, CT), (unsigned)nchunk);
    const int mi = (int)m;
    if (m <= 4)
        ht_kernel<1><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
    else if (m <= 8)
        ht_kernel<2><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
    else if (m <= 16)
        ht_kernel<4><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
    else
        ht_kernel<16><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
    ELM_LAUNCH_CHECK();
    ht_reduce_kernel<<<nred, NT, 0, s>>>(L, mi, nchunk, part, G, ldg, sq);
    ELM_LAUNCH_CHECK();
    sum_kernel<<<1, NT, 0, s>>>(nred, sq, nrm2);
    ELM_LAUNCH_CHECK();
}

void launch_axpy_mat(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy) {
    if (rows <= 0 || cols <= 0) return;
    axpy_mat_kernel<<<(unsigned)cdiv(rows * cols, 256), 256, 0, s>>>(rows, cols, X, ldx, Y, ldy);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
