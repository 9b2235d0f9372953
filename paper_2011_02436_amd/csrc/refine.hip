// FP64 streaming passes over the sample-major FP64 hidden matrix H (N x L)
// for the normal-equation residual of beta = H^+ T (eqs. 5 and 8):
//   E = T - H beta           residual_kernel  (one pass over H)
//   G = H^T E, ||G||_F^2      ht_kernel + ht_reduce_kernel (one pass over H)
// G with E = T is the right-hand side H^T T of eq. (8).  Every sum runs in a
// fixed order (no atomics), so repeated runs are bitwise identical.
#include "elm_internal.h"

#include <algorithm>

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
// rows_dot_kernel: out[row][o] = sign * (H beta)[row][o] + (T ? T[row][o] : 0).
//   Each wave owns RW rows (16 for m <= 4, else 32 / MM: up to 64 FP64
//   partial sums per lane);
//   lane l walks columns l, l + 64, ..., and a halving exchange across the
//   64 lanes forms the row sums (each by a butterfly's pairwise tree).  The order of every sum is fixed by the column stride
//   64 alone (not by the rows per wave or the launch), no LDS, no barrier.
//   H is read once per pass: its loads are non-temporal, so it does not push
//   beta (re-read by every wave) and the partials out of the caches.
//   With labels, also the arg-max of each row (lowest index on ties).
// cols_dot_kernel: part[chunk][col][o] = sum over the chunk's rows of
//   H[row][col] E[row][o], row by row; CPT columns per thread (more for wide
//   m, so that each E value read from LDS serves several columns), the
//   chunk's E rows in LDS.
// ---------------------------------------------------------------------------
constexpr int SB = 256;   // threads per block
constexpr int CR_ROWS = 1024;  // rows per chunk, cols_dot_kernel
template <int MM>
struct RowsDot {
    static constexpr int RW = MM <= 4 ? 16 : 32 / MM;  // rows per wave
    static constexpr int RB = RW * SB / 64;  // rows per block
};

template <int MM>
__device__ __forceinline__ void rows_dot_body(int64_t bx, int64_t N, int64_t L, int m,
                                     const double* __restrict__ H, int64_t ldh,
                                     const double* __restrict__ beta, int64_t ldb,
                                     const double* __restrict__ T, int64_t ldt, double sign,
                                     double* __restrict__ out, int64_t ldo,
                                     int32_t* __restrict__ labels, double* __restrict__ y,
                                     int64_t ldy) {
    constexpr int RW = RowsDot<MM>::RW;
    const int lane = threadIdx.x & 63;
    // the wave index is uniform: row addresses stay in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t r0 = bx * RowsDot<MM>::RB + (int64_t)wave * RW;
    if (r0 >= N) return;
    double acc[RW][MM];
#pragma unroll
    for (int r = 0; r < RW; ++r)
#pragma unroll
        for (int c = 0; c < MM; ++c) acc[r][c] = 0.0;
    const double* __restrict__ hrow[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) hrow[r] = H + min(r0 + r, N - 1) * ldh;
#pragma unroll 2
    for (int64_t col = lane; col < L; col += 64) {
        double bv[MM];
#pragma unroll
        for (int c = 0; c < MM; ++c) bv[c] = c < m ? beta[col * ldb + c] : 0.0;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const double h = __builtin_nontemporal_load(&hrow[r][col]);
#pragma unroll
            for (int c = 0; c < MM; ++c) acc[r][c] += h * bv[c];
        }
    }
    // Row sums by a halving exchange over the 64 lanes (offsets 32, 16, ..., 1):
    // at offset o a lane keeps half of its V partial sums (the upper half when
    // lane & o) and adds its partner's values of that half, V/2 + V/4 + ...
    // exchanges instead of 6 V.  Every sum is still formed by the pairwise
    // tree of a butterfly over that value alone (own + partner at each level),
    // so the results are those of one.  Value r MM + c ends in lane
    // (r MM + c) DUP.
    constexpr int V = RW * MM, DUP = 64 / V;
    static_assert(V <= 64 && (V & (V - 1)) == 0, "a power-of-two count of sums per lane");
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int o = 32 >> k, n = V >> k;
        if (n > 1) {
            const bool up = (lane & o) != 0;
#pragma unroll
            for (int i = 0; i < n / 2; ++i) {
                double& lo = acc[i / MM][i % MM];
                const double hi = acc[(i + n / 2) / MM][(i + n / 2) % MM];
                const double send = up ? lo : hi, keep = up ? hi : lo;
                lo = keep + __shfl_xor(send, o);
            }
        } else {
            acc[0][0] += __shfl_xor(acc[0][0], o);
        }
    }
    const double v = acc[0][0];
    const int idx = lane / DUP, rr = idx / MM, c = idx % MM;
    const int64_t row = r0 + rr;
    // one lane per value writes column c of its row
    if (lane % DUP == 0 && row < N && c < m) {
        if (out) out[row * ldo + c] = sign * v + (T ? T[row * ldt + c] : 0.0);
        if (y) y[row * ldy + c] = v;
    }
    if (labels) {
        // the row's values sit in lanes (rr MM + c') DUP; its column-0 lane
        // takes the arg-max (lowest index on ties)
        double vals[MM];
        vals[0] = v;
#pragma unroll
        for (int cc = 1; cc < MM; ++cc) vals[cc] = __shfl(v, (lane + cc * DUP) & 63);
        if (c == 0 && lane % DUP == 0 && row < N) {
            int best = 0;
            double bvv = vals[0];
#pragma unroll
            for (int cc = 1; cc < MM; ++cc)
                if (cc < m && vals[cc] > bvv) {
                    bvv = vals[cc];
                    best = cc;
                }
            labels[row] = best;
        }
    }
}

// Rows of a problem with 4 < m <= 16 on the FP64 16x16x4 MFMA (the wave
// form above reloads m values of beta per column and row group and then
// spends its time in the lane exchange).  A wave takes two groups of 16 rows
// (each beta value read serves both) and the 16 output columns (beta's
// columns past m read as zeros); in each group lane (r, q) =
// (lane % 16, lane / 16) reads H[row r][8 g + 2 q .. 8 g + 2 q + 1] as one
// 16-byte pair and feeds the two values to two steps, so every sum runs over
// the columns 8 g + 2 q, then 8 g + 2 q + 1, group after group, whatever the
// launch.  Row arg-max (lowest index on ties) over the 16 lanes of the row.
typedef double d2v __attribute__((ext_vector_type(2)));
constexpr int RMG = 2;                     // groups of 16 rows per wave (sharing beta's reads)
constexpr int RMB = 16 * RMG * (SB / 64);  // rows per block
__device__ __forceinline__ void rows_mfma_body(int64_t bx, int64_t N, int64_t L, int m,
                                               const double* __restrict__ H, int64_t ldh,
                                               const double* __restrict__ beta, int64_t ldb,
                                               const double* __restrict__ T, int64_t ldt, double sign,
                                               double* __restrict__ out, int64_t ldo,
                                               int32_t* __restrict__ labels, double* __restrict__ y,
                                               int64_t ldy) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t r0 = bx * RMB + (int64_t)wave * 16 * RMG;
    if (r0 >= N) return;
    const int q = lane >> 4, c = lane & 15;
    const double* __restrict__ hrow[RMG];  // A rows: lane % 16 of each group
    d4v acc[RMG];
#pragma unroll
    for (int g = 0; g < RMG; ++g) {
        hrow[g] = H + min(r0 + 16 * g + c, N - 1) * ldh;
        acc[g] = d4v{};
    }
    const bool cv = c < m;
    const int64_t L8 = L & ~(int64_t)7;
    // 16-byte pairs when every row starts 16-byte aligned (block-uniform)
    const bool pairs = ((((uintptr_t)H) | (uintptr_t)(ldh * 8)) & 15) == 0;
    int64_t k = 0;
    if (pairs) {
#pragma unroll 2
        for (; k < L8; k += 8) {
            d2v h[RMG];
#pragma unroll
            for (int g = 0; g < RMG; ++g) h[g] = *(const d2v*)(hrow[g] + k + 2 * q);
            const double b0 = cv ? beta[(k + 2 * q) * ldb + c] : 0.0;
            const double b1 = cv ? beta[(k + 2 * q + 1) * ldb + c] : 0.0;
#pragma unroll
            for (int g = 0; g < RMG; ++g) {
                acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[g].x, b0, acc[g], 0, 0, 0);
                acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(h[g].y, b1, acc[g], 0, 0, 0);
            }
        }
    } else {
#pragma unroll 2
        for (; k < L8; k += 8) {
            double h0[RMG], h1[RMG];
#pragma unroll
            for (int g = 0; g < RMG; ++g) {
                h0[g] = hrow[g][k + 2 * q];
                h1[g] = hrow[g][k + 2 * q + 1];
            }
            const double b0 = cv ? beta[(k + 2 * q) * ldb + c] : 0.0;
            const double b1 = cv ? beta[(k + 2 * q + 1) * ldb + c] : 0.0;
#pragma unroll
            for (int g = 0; g < RMG; ++g) {
                acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(h0[g], b0, acc[g], 0, 0, 0);
                acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(h1[g], b1, acc[g], 0, 0, 0);
            }
        }
    }
    if (k < L) {  // the last group, fewer than 8 columns (wave-uniform)
        const int64_t k0 = k + 2 * q, k1 = k0 + 1;
        const double b0 = (cv && k0 < L) ? beta[k0 * ldb + c] : 0.0;
        const double b1 = (cv && k1 < L) ? beta[k1 * ldb + c] : 0.0;
#pragma unroll
        for (int g = 0; g < RMG; ++g) {
            const double h0 = k0 < L ? hrow[g][k0] : 0.0, h1 = k1 < L ? hrow[g][k1] : 0.0;
            acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(h0, b0, acc[g], 0, 0, 0);
            acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(h1, b1, acc[g], 0, 0, 0);
        }
    }
#pragma unroll
    for (int g = 0; g < RMG; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = r0 + 16 * g + Mfma16<double>::row(lane, v);  // column c = lane % 16
            const double val = acc[g][v];
            if (row < N && cv) {
                if (out) out[row * ldo + c] = sign * val + (T ? T[row * ldt + c] : 0.0);
                if (y) y[row * ldy + c] = val;
            }
            if (labels) {
                double bv = cv ? val : -INFINITY;
                int bi = c;
#pragma unroll
                for (int o = 8; o > 0; o >>= 1) {
                    const double ov = __shfl_xor(bv, o);
                    const int oi = __shfl_xor(bi, o);
                    if (ov > bv || (ov == bv && oi < bi)) {
                        bv = ov;
                        bi = oi;
                    }
                }
                if (c == 0 && row < N) labels[row] = bi;
            }
        }
}

// columns per thread of cols_dot_kernel: each E value read from LDS serves
// CPT columns, so that a row costs about four LDS reads per H element (the
// batches' grouped launches keep one column per thread: their narrow
// problems would leave most of a wider block idle; a column's sum does not
// depend on it)
template <int MM>
struct ColsDot {
    static constexpr int CPT = MM >= 8 ? MM / 4 : 1;
    static constexpr int CB = SB * CPT;  // columns per block
};

// Rows per chunk of the column pass: CR_ROWS, and for an H of at least 2^26
// elements halved (down to 128) while the pass would have fewer than 512
// blocks (a function of the problem's own N, L and m, so a batch chunks each
// problem as its single training does).  On N = 60000, L = 2000, m = 10
// (118 blocks of 1024 rows) four passes took 2.0 ms, 1.65 in chunks of 128
// rows; a 1024-block bar also split N = 100000, L = 5000, m = 7 (980 blocks),
// whose partial sums then cost more than the blocks gained, and without the
// size floor the batch's small problems took their column passes from 12.6
// to 14.8 ms per 256 trainings.
__host__ __device__ inline int cols_rows(int64_t N, int64_t L, int m) {
    int cr = CR_ROWS;
    if (N * L < ((int64_t)1 << 26)) return cr;
    const int64_t cb = (int64_t)SB * (m > 8 ? 4 : m > 4 ? 2 : 1);
    const int64_t nbx = (L + cb - 1) / cb;
    while (cr > 128 && nbx * ((N + cr - 1) / cr) < 512) cr >>= 1;
    return cr;
}

template <int MM, int CPT = ColsDot<MM>::CPT, int CRCAP = CR_ROWS>
__device__ __forceinline__ void cols_dot_body(int64_t bx, int64_t by, int64_t N, int64_t L, int m,
                                     const double* __restrict__ H, int64_t ldh,
                                     const double* __restrict__ E, int64_t lde,
                                     double* __restrict__ part) {
    constexpr int RU = CPT > 2 ? 4 : 8;  // rows per unrolled step
    __shared__ double Es[CRCAP * MM];  // the chunk's rows of E (cr <= CRCAP)
    const int tid = threadIdx.x;
    // thread columns col0 + j SB, j < CPT (each load instruction reads 64
    // consecutive columns); a column past L reads column L - 1, unstored
    const int64_t col0 = bx * (SB * CPT) + tid;
    const int cr = cols_rows(N, L, m);
    const int64_t rbeg = by * cr;
    const int nrows = (int)min<int64_t>(cr, N - rbeg);
    for (int e = tid; e < cr * MM; e += SB) {
        const int r = e / MM, c = e % MM;
        Es[e] = (r < nrows && c < m) ? E[(rbeg + r) * lde + c] : 0.0;
    }
    __syncthreads();
    if (col0 >= L) return;  // no barrier follows
    double acc[CPT][MM];
    const double* __restrict__ hp[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
#pragma unroll
        for (int c = 0; c < MM; ++c) acc[j][c] = 0.0;
        hp[j] = H + rbeg * ldh + min(col0 + (int64_t)j * SB, L - 1);
    }
    int r = 0;
    for (; r + RU <= nrows; r += RU) {
        double h[RU][CPT];
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int j = 0; j < CPT; ++j) h[u][j] = __builtin_nontemporal_load(&hp[j][(int64_t)(r + u) * ldh]);
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int c = 0; c < MM; ++c) {
                const double e = Es[(r + u) * MM + c];
#pragma unroll
                for (int j = 0; j < CPT; ++j) acc[j][c] += h[u][j] * e;
            }
    }
    for (; r < nrows; ++r) {
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const double hv = __builtin_nontemporal_load(&hp[j][(int64_t)r * ldh]);
#pragma unroll
            for (int c = 0; c < MM; ++c) acc[j][c] += hv * Es[r * MM + c];
        }
    }
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int64_t col = col0 + (int64_t)j * SB;
        if (col >= L) continue;
        double* o = part + by * L * m + col * m;
#pragma unroll
        for (int c = 0; c < MM; ++c)
            if (c < m) o[c] = acc[j][c];
    }
}

// G[i][o] = sum over chunks of the partials; per-block sum of squares
__device__ __forceinline__ void ht_reduce_body(int64_t bx, int64_t L, int m, int nchunk,
                                      const double* __restrict__ part, double* __restrict__ G,
                                      int64_t ldg, double* __restrict__ sq_part) {
    const int64_t e = bx * NT + threadIdx.x;
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
    if (threadIdx.x == 0) sq_part[bx] = red[0];
}

__device__ __forceinline__ void sum_body(int64_t n, const double* __restrict__ x, double* __restrict__ out) {
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

// Y += X; the previous Y is kept in B (ld cols), so that a correction that
// did not lower the residual can be taken back exactly.
__device__ __forceinline__ void axpy_mat_body(int64_t bx, int64_t rows, int64_t cols,
                                     const double* __restrict__ X, int64_t ldx,
                                     double* __restrict__ Y, int64_t ldy,
                                     double* __restrict__ B) {
    const int64_t e = bx * blockDim.x + threadIdx.x;
    if (e < rows * cols) {
        const int64_t i = e / cols, j = e % cols;
        const double y = Y[i * ldy + j];
        B[e] = y;
        Y[i * ldy + j] = y + X[i * ldx + j];
    }
}

template <int MM>
__global__ __launch_bounds__(SB, 2) void rows_dot_kernel(int64_t N, int64_t L, int m,
                                                      const double* __restrict__ H, int64_t ldh,
                                                      const double* __restrict__ beta, int64_t ldb,
                                                      const double* __restrict__ T, int64_t ldt,
                                                      double sign, double* __restrict__ out,
                                                      int64_t ldo, int32_t* __restrict__ labels,
                                                      double* __restrict__ y, int64_t ldy) {
    if constexpr (MM > 4)
        rows_mfma_body(blockIdx.x, N, L, m, H, ldh, beta, ldb, T, ldt, sign, out, ldo, labels, y, ldy);
    else
        rows_dot_body<MM>(blockIdx.x, N, L, m, H, ldh, beta, ldb, T, ldt, sign, out, ldo, labels, y,
                          ldy);
}

// CRCAP: the largest chunk the launch may take; a launch whose chunks are
// 128 rows reserves that much LDS, so more blocks share a CU
template <int MM, int CRCAP>
__global__ __launch_bounds__(SB) void cols_dot_kernel(int64_t N, int64_t L, int m,
                                                      const double* __restrict__ H, int64_t ldh,
                                                      const double* __restrict__ E, int64_t lde,
                                                      double* __restrict__ part) {
    cols_dot_body<MM, ColsDot<MM>::CPT, CRCAP>(blockIdx.x, blockIdx.y, N, L, m, H, ldh, E, lde, part);
}

__global__ __launch_bounds__(NT) void ht_reduce_kernel(int64_t L, int m, int nchunk,
                                                       const double* __restrict__ part,
                                                       double* __restrict__ G, int64_t ldg,
                                                       double* __restrict__ sq_part) {
    ht_reduce_body(blockIdx.x, L, m, nchunk, part, G, ldg, sq_part);
}

__global__ __launch_bounds__(NT) void sum_kernel(int64_t n, const double* __restrict__ x,
                                                 double* __restrict__ out) {
    sum_body(n, x, out);
}

__global__ void axpy_mat_kernel(int64_t rows, int64_t cols, const double* __restrict__ X,
                                int64_t ldx, double* __restrict__ Y, int64_t ldy,
                                double* __restrict__ B) {
    axpy_mat_body(blockIdx.x, rows, cols, X, ldx, Y, ldy, B);
}

// ---------------------------------------------------------------------------
// Grouped refinement passes: one launch serves every scheduled problem of a
// batch.  The launch's blocks are laid out problem after problem (GroupSched);
// each block runs the single-problem kernel's body with that problem's
// arguments and its own block index, so the arithmetic is the same.
// ---------------------------------------------------------------------------
template <int MM>
__global__ __launch_bounds__(SB, 2) void rows_dot_grouped(const RefineDesc* __restrict__ d,
                                                       GroupSched g) {
    int64_t lb;
    const int j = group_problem(g, lb);
    if (!group_live(g, j)) return;
    const RefineDesc& q = d[j];
    // the form of the problem's own m (that of its single training)
    if (MM > 4 && q.m > 4)
        rows_mfma_body(lb, q.N, q.L, q.m, q.H, q.ldh, q.beta, q.ldbeta, q.T, q.ldt, -1.0, q.E, q.m,
                       nullptr, nullptr, 0);
    else
        rows_dot_body<MM>(lb, q.N, q.L, q.m, q.H, q.ldh, q.beta, q.ldbeta, q.T, q.ldt, -1.0, q.E, q.m,
                          nullptr, nullptr, 0);
}

template <int MM>
__global__ __launch_bounds__(SB) void cols_dot_grouped(const RefineDesc* __restrict__ d,
                                                       GroupSched g) {
    int64_t lb;
    const int j = group_problem(g, lb);
    if (!group_live(g, j)) return;
    const RefineDesc& q = d[j];
    const int64_t nbx = cdiv(q.L, SB);
    cols_dot_body<MM, 1>(lb % nbx, lb / nbx, q.N, q.L, q.m, q.H, q.ldh, q.E, q.m, q.part);
}

__global__ __launch_bounds__(NT) void ht_reduce_grouped(const RefineDesc* __restrict__ d,
                                                        GroupSched g) {
    int64_t lb;
    const int j = group_problem(g, lb);
    if (!group_live(g, j)) return;
    const RefineDesc& q = d[j];
    ht_reduce_body(lb, q.L, q.m, (int)cdiv(q.N, cols_rows(q.N, q.L, q.m)), q.part, q.G, q.m, q.sq);
}

__global__ __launch_bounds__(NT) void sum_grouped(const RefineDesc* __restrict__ d, GroupSched g) {
    int64_t lb;
    const int j = group_problem(g, lb);
    if (!group_live(g, j)) return;
    const RefineDesc& q = d[j];
    sum_body(cdiv(q.L * q.m, NT), q.sq, q.g2);
}

__global__ void axpy_grouped(const RefineDesc* __restrict__ d, GroupSched g) {
    int64_t lb;
    const int j = group_problem(g, lb);
    if (!group_live(g, j)) return;
    const RefineDesc& q = d[j];
    axpy_mat_body(lb, q.L, q.m, q.D, q.m, q.beta, q.ldbeta, q.prev);
}

__global__ void restore_grouped(const RefineDesc* __restrict__ d, GroupSched g) {
    int64_t lb;
    const int j = group_problem(g, lb);
    if (!group_live(g, j)) return;
    const RefineDesc& q = d[j];
    const int64_t e = lb * blockDim.x + threadIdx.x;
    if (e < q.L * q.m) {
        const int64_t i = e / q.m, c = e % q.m;
        q.beta[i * q.ldbeta + c] = q.prev[e];
    }
}

__global__ void ir_init_kernel(int P, IrCtl* __restrict__ c, int32_t* __restrict__ active,
                               int32_t* __restrict__ rollback) {
    for (int j = threadIdx.x; j < P; j += blockDim.x) {
        c[j] = IrCtl{};
        c[j].active = 1;
        active[j] = 1;
        rollback[j] = 0;
    }
}

// the single-problem loop's rules, one thread per problem
__global__ __launch_bounds__(256) void ir_decide_kernel(int P, IrCtl* __restrict__ c,
                                                        const RefineDesc* __restrict__ d,
                                                        int32_t* __restrict__ active,
                                                        int32_t* __restrict__ rollback,
                                                        int32_t* __restrict__ any, double tol,
                                                        int max_iter) {
    __shared__ int32_t live;
    if (threadIdx.x == 0) live = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < P; j += blockDim.x) {
        rollback[j] = 0;
        IrCtl& q = c[j];
        if (!q.active) continue;
        q.evals += 1;
        const double g2 = *d[j].g2, z2 = *d[j].z2;
        double res = z2 > 0 ? sqrt(g2 / z2) : sqrt(g2);
        if (q.it < 32) q.hist[q.it] = res;
        if (q.it >= 1 && !(res < q.prev)) {
            // no progress: stop, and take a diverging correction back
            if (!(res <= IR_RISE * q.prev)) {
                rollback[j] = 1;
                q.it -= 1;
                res = q.prev;
            }
            q.active = 0;
        } else if ((q.it >= 1 && !(res > tol)) || q.it >= max_iter) {
            q.active = 0;
        } else {
            q.prev = res;   // a correction follows
            q.it += 1;
        }
        q.res = res;
        active[j] = q.active;
        if (q.active) atomicOr(&live, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *any = live;
}

}  // namespace

void launch_ir_init(hipStream_t s, int P, IrCtl* c, int32_t* active, int32_t* rollback) {
    ir_init_kernel<<<1, 256, 0, s>>>(P, c, active, rollback);
    ELM_LAUNCH_CHECK();
}

void launch_ir_decide(hipStream_t s, int P, IrCtl* c, const RefineDesc* d, int32_t* active,
                      int32_t* rollback, int32_t* any, double ir_tol, int ir_max_iter) {
    ir_decide_kernel<<<1, 256, 0, s>>>(P, c, d, active, rollback, any, ir_tol, ir_max_iter);
    ELM_LAUNCH_CHECK();
}

void launch_restore_grouped(hipStream_t s, const RefineDesc* d, const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    restore_grouped<<<(unsigned)g.blocks, 256, 0, s>>>(d, g);
    ELM_LAUNCH_CHECK();
}

int64_t refine_group_blocks(RefinePass pass, const RefineDesc& q, int maxm) {
    switch (pass) {
        case RefinePass::ROWS_DOT:
            if (q.m > 4) return cdiv(q.N, RMB);
            return cdiv(q.N, maxm <= 2 ? RowsDot<2>::RB
                             : maxm <= 4 ? RowsDot<4>::RB
                             : maxm <= 8 ? RowsDot<8>::RB : RowsDot<16>::RB);
        case RefinePass::COLS_DOT: return cdiv(q.L, SB) * cdiv(q.N, cols_rows(q.N, q.L, (int)q.m));
        case RefinePass::HT_REDUCE: return cdiv(q.L * q.m, NT);
        case RefinePass::SUM: return 1;
        case RefinePass::AXPY: return cdiv(q.L * q.m, 256);
    }
    return 0;
}

size_t refine_part_doubles(int64_t N, int64_t L, int64_t m) {
    return (size_t)cdiv(N, cols_rows(N, L, (int)m)) * L * m;
}
size_t refine_sq_doubles(int64_t L, int64_t m) { return (size_t)cdiv(L * m, NT); }

void launch_refine_grouped(hipStream_t s, RefinePass pass, const RefineDesc* d, const GroupSched& g,
                           int maxm) {
    if (g.count <= 0 || g.blocks <= 0) return;
    const unsigned grid = (unsigned)g.blocks;
    switch (pass) {
        case RefinePass::ROWS_DOT:
        case RefinePass::COLS_DOT: {
#define ELM_RG(MM)                                                                   \
    do {                                                                             \
        if (pass == RefinePass::ROWS_DOT)                                            \
            rows_dot_grouped<MM><<<grid, SB, 0, s>>>(d, g);                          \
        else                                                                         \
            cols_dot_grouped<MM><<<grid, SB, 0, s>>>(d, g);                          \
    } while (0)
            if (maxm <= 2) ELM_RG(2);
            else if (maxm <= 4) ELM_RG(4);
            else if (maxm <= 8) ELM_RG(8);
            else if (maxm <= 16) ELM_RG(16);
            else throw Error{ELM_ERR_UNSUPPORTED, "grouped refinement needs m <= 16"};
#undef ELM_RG
            break;
        }
        case RefinePass::HT_REDUCE: ht_reduce_grouped<<<grid, NT, 0, s>>>(d, g); break;
        case RefinePass::SUM: sum_grouped<<<grid, NT, 0, s>>>(d, g); break;
        case RefinePass::AXPY: axpy_grouped<<<grid, 256, 0, s>>>(d, g); break;
    }
    ELM_LAUNCH_CHECK();
}

static void launch_rows_dot(hipStream_t s, int64_t N, int64_t L, int64_t m, const double* H,
                            int64_t ldh, const double* beta, int64_t ldb, const double* T, int64_t ldt,
                            double sign, double* out, int64_t ldo, int32_t* labels,
                            double* y = nullptr, int64_t ldy = 0) {
    const int mi = (int)m;
#define ELM_RD(MM)                                                                                  \
    rows_dot_kernel<MM><<<(unsigned)cdiv(N, MM > 4 ? RMB : RowsDot<MM>::RB), SB, 0, s>>>(           \
        N, L, mi, H, ldh, beta, ldb, T, ldt, sign, out, ldo, labels, y, ldy)
    if (m <= 2)
        ELM_RD(2);
    else if (m <= 4)
        ELM_RD(4);
    else if (m <= 8)
        ELM_RD(8);
    else if (m <= 16)
        ELM_RD(16);
    else
        throw Error{ELM_ERR_UNSUPPORTED, "m > 16 on the streaming row pass"};
#undef ELM_RD
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
__device__ __forceinline__ void group_sum_body(int64_t bx, int64_t by, int64_t len, int64_t nchunk,
                                               int gs, const double* __restrict__ part,
                                               double* __restrict__ out) {
    const int64_t e = bx * NT + threadIdx.x;
    if (e >= len) return;
    const int64_t c0 = by * gs;
    const int64_t c1 = c0 + gs < nchunk ? c0 + gs : nchunk;
    double acc = 0.0;
    for (int64_t c = c0; c < c1; ++c) acc += part[c * len + e];
    out[by * len + e] = acc;
}

__global__ __launch_bounds__(NT) void group_sum_kernel(int64_t len, int64_t nchunk, int gs,
                                                       const double* __restrict__ part,
                                                       double* __restrict__ out) {
    group_sum_body(blockIdx.x, blockIdx.y, len, nchunk, gs, part, out);
}

constexpr int PSUM_GS = 64;  // chunks per group sum (two levels above 2 PSUM_GS chunks)

// launch_partial_sum of a batch: stage 0 the group sums, 1 the column sums
// and their squares, 2 the total
template <int STAGE>
__global__ __launch_bounds__(NT) void partial_sum_grouped(const PsumDesc* __restrict__ d,
                                                          GroupSched g) {
    int64_t lb;
    const PsumDesc& q = d[group_problem(g, lb)];
    const int64_t len = q.L * q.m;
    const bool two = q.nchunk > 2 * PSUM_GS;
    if constexpr (STAGE == 0) {
        const int64_t nbx = cdiv(len, NT);
        group_sum_body(lb % nbx, lb / nbx, len, q.nchunk, PSUM_GS, q.part, q.part2);
    } else if constexpr (STAGE == 1) {
        ht_reduce_body(lb, q.L, (int)q.m, (int)(two ? cdiv(q.nchunk, PSUM_GS) : q.nchunk),
                       two ? q.part2 : q.part, q.G, q.m, q.sq);
    } else {
        sum_body(cdiv(len, NT), q.sq, q.nrm2);
    }
}

size_t psum_part2_doubles(int64_t L, int64_t m, int64_t nchunk) {
    return nchunk > 2 * PSUM_GS ? (size_t)cdiv(nchunk, PSUM_GS) * L * m : 0;
}

int64_t partial_sum_group_blocks(int stage, const PsumDesc& q) {
    const int64_t len = q.L * q.m;
    if (stage == 0) return q.nchunk > 2 * PSUM_GS ? cdiv(len, NT) * cdiv(q.nchunk, PSUM_GS) : 0;
    if (stage == 1) return cdiv(len, NT);
    return 1;
}

void launch_partial_sum_grouped(hipStream_t s, int stage, const PsumDesc* d, const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    const unsigned grid = (unsigned)g.blocks;
    if (stage == 0)
        partial_sum_grouped<0><<<grid, NT, 0, s>>>(d, g);
    else if (stage == 1)
        partial_sum_grouped<1><<<grid, NT, 0, s>>>(d, g);
    else
        partial_sum_grouped<2><<<grid, NT, 0, s>>>(d, g);
    ELM_LAUNCH_CHECK();
}

void launch_partial_sum(hipStream_t s, int64_t L, int64_t m, int64_t nchunk, const double* part,
                        double* G, int64_t ldg, double* nrm2, Workspace& ws) {
    constexpr int GS = PSUM_GS;
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
        const int cr = cols_rows(N, L, mi);
        nchunk = (int)cdiv(N, cr);
        part = (double*)ws.get("ht_part", (size_t)nchunk * L * m * sizeof(double));
#define ELM_CD(MM)                                                                               \
    do {                                                                                         \
        const dim3 grid((unsigned)cdiv(L, ColsDot<MM>::CB), (unsigned)nchunk);                   \
        if (cr <= 128)                                                                           \
            cols_dot_kernel<MM, 128><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, E, lde, part);        \
        else                                                                                     \
            cols_dot_kernel<MM, CR_ROWS><<<grid, SB, 0, s>>>(N, L, mi, H, ldh, E, lde, part);    \
    } while (0)
        if (m <= 2)
            ELM_CD(2);
        else if (m <= 4)
            ELM_CD(4);
        else if (m <= 8)
            ELM_CD(8);
        else
            ELM_CD(16);
#undef ELM_CD
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

__global__ void add_mat_kernel(int64_t rows, int64_t cols, const double* __restrict__ X, int64_t ldx,
                               double* __restrict__ Y, int64_t ldy) {
    const int64_t i = blockIdx.y;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cols;
         j += (int64_t)gridDim.x * blockDim.x)
        Y[i * ldy + j] += X[i * ldx + j];
}

void launch_add_mat(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx, double* Y,
                    int64_t ldy) {
    if (rows <= 0 || cols <= 0) return;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(cols, 256), 64);
    for (int64_t r0 = 0; r0 < rows; r0 += 65535) {
        const int64_t nr = std::min<int64_t>(65535, rows - r0);
        add_mat_kernel<<<dim3(gx, (unsigned)nr), 256, 0, s>>>(nr, cols, X + r0 * ldx, ldx, Y + r0 * ldy, ldy);
        ELM_LAUNCH_CHECK();
    }
}

// Y += X (rows x cols); prev (rows x cols, ld cols) receives the old Y, so a
// correction that did not lower the residual can be taken back.
void launch_axpy_mat(hipStream_t s, int64_t rows, int64_t cols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy, double* prev) {
    if (rows <= 0 || cols <= 0) return;
    axpy_mat_kernel<<<(unsigned)cdiv(rows * cols, 256), 256, 0, s>>>(rows, cols, X, ldx, Y, ldy,
                                                                      prev);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
