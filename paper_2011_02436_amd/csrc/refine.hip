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

// Y = H beta and/or the arg-max label per row (lowest index on ties), from a
// stored sample-major H: step 3 of the three-step ELM.  Same tiling as
// residual_kernel.
template <int OPT>
__global__ __launch_bounds__(NT) void hidden_output_kernel(int64_t N, int64_t L, int m,
                                                           const double* __restrict__ H, int64_t ldh,
                                                           const double* __restrict__ beta, int64_t ldb,
                                                           double* __restrict__ Y, int64_t ldy,
                                                           int32_t* __restrict__ labels) {
    __shared__ double Hs[RT][CT + 1];
    __shared__ double Bs[CT][4 * OPT];
    __shared__ double Ys[RT][4 * OPT];
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
#pragma unroll
    for (int j = 0; j < OPT; ++j) Ys[row][grp + 4 * j] = acc[j];
    __syncthreads();
    const int64_t gi = n0 + row;
    if (gi >= N) return;
    if (Y)
#pragma unroll
        for (int j = 0; j < OPT; ++j) {
            const int o = grp + 4 * j;
            if (o < m) Y[gi * ldy + o] = acc[j];
        }
    if (labels && grp == 0) {
        int best = 0;
        double bv = Ys[row][0];
        for (int o = 1; o < m; ++o)
            if (Ys[row][o] > bv) { bv = Ys[row][o]; best = o; }
        labels[gi] = best;
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


// ---------------------------------------------------------------------------
// Streaming passes built for HBM bandwidth.
//
// rows_dot_kernel: out[row][o] = sign * (H beta)[row][o] + (T ? T[row][o] : 0)
//   for RB rows per block; thread t walks columns t, t + 256, ... keeping
//   RB x MM partial sums, so each beta row it loads (through the cache) serves
//   RB rows of H; one block reduction at the end.  With labels, also the
//   arg-max of each row (lowest index on ties).
// cols_dot_kernel: part[chunk][col][o] = sum over the chunk's rows of
//   H[row][col] E[row][o]; thread per column, the chunk's E rows in LDS.
// ---------------------------------------------------------------------------
constexpr int SB = 256;   // threads per block
constexpr int RBR = 8;    // rows per block, rows_dot_kernel
constexpr int CR_ROWS = 1024;  // rows per chunk, cols_dot_kernel

template <int MM>
__global__ __launch_bounds__(SB) void rows_dot_kernel(int64_t N, int64_t L, int m,
                                                      const double* __restrict__ H, int64_t ldh,
                                                      const double* __restrict__ beta, int64_t ldb,
                                                      const double* __restrict__ T, int64_t ldt,
                                                      double sign, double* __restrict__ out,
                                                      int64_t ldo, int32_t* __restrict__ labels,
                                                      double* __restrict__ y, int64_t ldy) {
    __shared__ double red[SB / 64][RBR * MM];
    __shared__ double fin[RBR * MM];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * RBR;
    double acc[RBR][MM];
#pragma unroll
    for (int r = 0; r < RBR; ++r)
#pragma unroll
        for (int c = 0; c < MM; ++c) acc[r][c] = 0.0;
    const double* __restrict__ hrow[RBR];
#pragma unroll
    for (int r = 0; r < RBR; ++r) hrow[r] = H + min(r0 + r, N - 1) * ldh;
    for (int64_t col = tid; col < L; col += SB) {
        double bv[MM];
#pragma unroll
        for (int c = 0; c < MM; ++c) bv[c] = c < m ? beta[col * ldb + c] : 0.0;
#pragma unroll
        for (int r = 0; r < RBR; ++r) {
            const double h = hrow[r][col];
#pragma unroll
            for (int c = 0; c < MM; ++c) acc[r][c] += h * bv[c];
        }
    }
#pragma unroll
    for (int r = 0; r < RBR; ++r)
#pragma unroll
        for (int c = 0; c < MM; ++c) {
            double v = acc[r][c];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) red[wave][r * MM + c] = v;
        }
    __syncthreads();
    if (tid < RBR * MM) {
        double v = 0.0;
        for (int w = 0; w < SB / 64; ++w) v += red[w][tid];
        const int r = tid / MM, c = tid % MM;
        const int64_t row = r0 + r;
        double o = sign * v;
        if (T && row < N && c < m) o += T[row * ldt + c];
        fin[tid] = v;
        if (out && row < N && c < m) out[row * ldo + c] = o;
        if (y && row < N && c < m) y[row * ldy + c] = v;
    }
    if (labels) {
        __syncthreads();
        if (tid < RBR && r0 + tid < N) {
            int best = 0;
            double bvv = fin[tid * MM];
            for (int c = 1; c < m; ++c)
                if (fin[tid * MM + c] > bvv) { bvv = fin[tid * MM + c]; best = c; }
            labels[r0 + tid] = best;
        }
    }
}

template <int MM>
__global__ __launch_bounds__(SB) void cols_dot_kernel(int64_t N, int64_t L, int m,
                                                      const double* __restrict__ H, int64_t ldh,
                                                      const double* __restrict__ E, int64_t lde,
                                                      double* __restrict__ part) {
    __shared__ double Es[CR_ROWS * MM];
    const int tid = threadIdx.x;
    const int64_t col = (int64_t)blockIdx.x * SB + tid;
    const int64_t rbeg = (int64_t)blockIdx.y * CR_ROWS;
    const int nrows = (int)min<int64_t>(CR_ROWS, N - rbeg);
    for (int e = tid; e < CR_ROWS * MM; e += SB) {
        const int r = e / MM, c = e % MM;
        Es[e] = (r < nrows && c < m) ? E[(rbeg + r) * lde + c] : 0.0;
    }
    __syncthreads();
    double acc[MM];
#pragma unroll
    for (int c = 0; c < MM; ++c) acc[c] = 0.0;
    if (col < L) {
        const double* __restrict__ hp = H + rbeg * ldh + col;
        int r = 0;
        for (; r + 8 <= nrows; r += 8) {
            double h[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) h[u] = hp[(int64_t)(r + u) * ldh];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < MM; ++c) acc[c] += h[u] * Es[(r + u) * MM + c];
        }
        for (; r < nrows; ++r) {
            const double hv = hp[(int64_t)r * ldh];
#pragma unroll
            for (int c = 0; c < MM; ++c) acc[c] += hv * Es[r * MM + c];
        }
        double* o = part + (int64_t)blockIdx.y * L * m + col * m;
#pragma unroll
        for (int c = 0; c < MM; ++c)
            if (c < m) o[c] = acc[c];
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

static void launch_rows_dot(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H,
                            int64_t ldh, const double* beta, int64_t ldb, const double* T, int64_t ldt,
                            double sign, double* out, int64_t ldo, int32_t* labels,
                            double* y = nullptr, int64_t ldy = 0) {
    const unsigned grid = (unsigned)cdiv(N, RBR);
    const int mi = (int)m;
    if (m <= 2)
        rows_dot_kernel<2><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, beta, ldb, T, ldt, sign, out, ldo, labels, y, ldy);
    else if (m <= 4)
        rows_dot_kernel<4><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, beta, ldb, T, ldt, sign, out, ldo, labels, y, ldy);
    else if (m <= 8)
        rows_dot_kernel<8><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, beta, ldb, T, ldt, sign, out, ldo, labels, y, ldy);
    else if (m <= 16)
        rows_dot_kernel<16><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, beta, ldb, T, ldt, sign, out, ldo, labels, y, ldy);
    else
        throw Error{ELM_ERR_UNSUPPORTED, "m > 16 on the streaming row pass"};
    ELM_LAUNCH_CHECK();
}

void launch_residual(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H, int64_t ldh,
                     const double* T, int64_t ldt, const double* beta, int64_t ldb, double* E,
                     int64_t lde, double* Y, int64_t ldy, int32_t* labels) {
    if (m <= 16) {
        launch_rows_dot(s, N, L, m, H, ldh, beta, ldb, T, ldt, -1.0, E, lde, labels, Y, ldy);
        return;
    }
    if (Y || labels) throw Error{ELM_ERR_UNSUPPORTED, "training outputs from the residual pass need m <= 16"};
    const unsigned grid = (unsigned)cdiv(N, RT);
    residual_kernel<16><<<grid, NT, 0, s>>>(N, L, (int)m, H, ldh, T, ldt, beta, ldb, E, lde);
    ELM_LAUNCH_CHECK();
}

void launch_hidden_output(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H,
                          int64_t ldh, const double* beta, int64_t ldb, double* Y, int64_t ldy,
                          int32_t* labels) {
    if (m <= 16) {
        launch_rows_dot(s, N, L, m, H, ldh, beta, ldb, nullptr, 0, 1.0, Y, ldy, labels);
        return;
    }
    const unsigned grid = (unsigned)cdiv(N, RT);
    hidden_output_kernel<16><<<grid, NT, 0, s>>>(N, L, (int)m, H, ldh, beta, ldb, Y, ldy, labels);
    ELM_LAUNCH_CHECK();
}

// out[g][e] = sum of part[c][e] over the chunks c of group g (GS consecutive
// chunks), in order
__global__ __launch_bounds__(NT) void group_sum_kernel(int64_t len, int64_t nchunk, int gs,
                                                       const double* __restrict__ part,
                                                       double* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= len) return;
    const int64_t c0 = (int64_t)blockIdx.y * gs;
    const int64_t c1 = c0 + gs < nchunk ? c0 + gs : nchunk;
    double acc = 0.0;
    for (int64_t c = c0; c < c1; ++c) acc += part[c * len + e];
    out[(int64_t)blockIdx.y * len + e] = acc;
}

void launch_partial_sum(hipStream_t s, int64_t L, int64_t m, int64_t nchunk, const double* part,
                        double* G, int64_t ldg, double* nrm2, Workspace& ws) {
    constexpr int GS = 64;
    if (nchunk > 2 * GS) {  // two levels, so that no thread sums thousands of chunks
        const int64_t ng = cdiv(nchunk, GS);
        double* part2 = (double*)ws.get("psum_part2", (size_t)ng * L * m * sizeof(double));
        group_sum_kernel<<<dim3((unsigned)cdiv(L * m, NT), (unsigned)ng), NT, 0, s>>>(L * m, nchunk, GS,
                                                                                    part, part2);
        ELM_LAUNCH_CHECK();
        part = part2;
        nchunk = ng;
    }
    const unsigned nred = (unsigned)cdiv(L * m, NT);
    double* sq = (double*)ws.get("ht_sq", (size_t)nred * sizeof(double));
    ht_reduce_kernel<<<nred, NT, 0, s>>>(L, (int)m, (int)nchunk, part, G, ldg, sq);
    ELM_LAUNCH_CHECK();
    sum_kernel<<<1, NT, 0, s>>>(nred, sq, nrm2);
    ELM_LAUNCH_CHECK();
}

void launch_ht_times(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H, int64_t ldh,
                     const double* E, int64_t lde, double* G, int64_t ldg, double* nrm2,
                     Workspace& ws) {
    const unsigned nred = (unsigned)cdiv(L * m, NT);
    double* sq = (double*)ws.get("ht_sq", (size_t)nred * sizeof(double));
    const int mi = (int)m;
    int nchunk;
    double* part;
    if (m <= 16) {
        nchunk = (int)cdiv(N, CR_ROWS);
        part = (double*)ws.get("ht_part", (size_t)nchunk * L * m * sizeof(double));
        dim3 grid((unsigned)cdiv(L, SB), (unsigned)nchunk);
        if (m <= 2)
            cols_dot_kernel<2><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
        else if (m <= 4)
            cols_dot_kernel<4><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
        else if (m <= 8)
            cols_dot_kernel<8><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
        else
            cols_dot_kernel<16><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
    } else {
        nchunk = (int)cdiv(N, HT_ROWS);
        part = (double*)ws.get("ht_part", (size_t)nchunk * L * m * sizeof(double));
        dim3 grid((unsigned)cdiv(L, CT), (unsigned)nchunk);
        ht_kernel<16><<<grid, NT, 0, s>>>(N, L, mi, H, ldh, E, lde, part);
    }
    ELM_LAUNCH_CHECK();
    ht_reduce_kernel<<<nred, NT, 0, s>>>(L, mi, nchunk, part, G, ldg, sq);
    ELM_LAUNCH_CHECK();
    sum_kernel<<<1, NT, 0, s>>>(nred, sq, nrm2);
    ELM_LAUNCH_CHECK();
}

// G = H^T (T - H beta) in one pass over H (beta = NULL: G = H^T T).
// Returns false when L or m is beyond what the register-resident partials hold.

void launch_axpy_mat(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy) {
    if (rows <= 0 || cols <= 0) return;
    axpy_mat_kernel<<<(unsigned)cdiv(rows * cols, 256), 256, 0, s>>>(rows, cols, X, ldx, Y, ldy);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
