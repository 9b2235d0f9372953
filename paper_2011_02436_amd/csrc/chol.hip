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
//   potrf_block   one workgroup: the block's Cholesky factor, panel by
//                 panel in LDS (one wave's register steps per 16 x 16
//                 diagonal block, MFMA tiles for the rest), written to U,
//                 then its inverse, written to W
//   copy          the block rows right of the diagonal block into T
//   product       U12 = W^T T                           (FP64 MFMA GEMM)
// and per group: S -= U_g^T U_g on the trailing matrix's upper tiles, with
// U_g the group's GB rows (FP64 MFMA GEMM, GB deep).
// A block that meets a pivot <= thr sets a device flag, and every later
// kernel returns at once.
#include "elm_internal.h"

#include <algorithm>
#include <cstring>
#include <functional>
#include <cmath>

namespace elm {
namespace {

constexpr int CB = 128;    // diagonal block
constexpr int GB = 2 * CB; // block rows per trailing update
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

// acc += A(r, k) B(k, c) over k in [0, K) for one 16 x 16 tile, with A and B
// read through accessors (all operand reads issued before the MFMAs); in the
// result, register v of lane l is row 4 v + l / 16, column l % 16
// (Mfma16<double>)
template <int K, typename FA, typename FB>
__device__ __forceinline__ d4v mma16_f64(d4v acc, int lane, FA fa, FB fb) {
    const int r = lane & 15, kq = lane >> 4;
    double av[K / 4], bv[K / 4];
#pragma unroll
    for (int s = 0; s < K / 4; ++s) {
        av[s] = fa(r, 4 * s + kq);
        bv[s] = fb(4 * s + kq, r);
    }
#pragma unroll
    for (int s = 0; s < K / 4; ++s) acc = Mfma16<double>::op(av[s], bv[s], acc);
    return acc;
}

constexpr int PW = 16;      // panel of the block factorisation
typedef double d2v __attribute__((ext_vector_type(2)));
constexpr int TS = PW / 8;  // elements per side of a lane's tile in the panel wave

// The CB x CB block is factored in LDS, one panel of PW rows at a time:
//   1. one wave factors the panel's PW x PW diagonal block D = U_pp^T U_pp
//      in registers (lane (rg, cg) of an 8 x 8 grid holds the TS x TS
//      elements rows TS rg .., columns TS cg ..), PW dependent steps with no
//      block barrier: step j reads its pivot from the diagonal owner
//      (readlane), publishes row j of U_pp in LDS and applies it to the
//      trailing elements.  The same steps build W_pp = U_pp^-1 by columns:
//      with S[i][c] = sum_{k < j} W[i][k] U[k][c] kept up to date, column j
//      of W is (e_j - S[:, j]) / U[j][j], and S then takes W[:, j] U[j][c].
//   2. the panel's rows right of D: U_pq = W_pp^T A_pq (FP64 MFMA tiles);
//   3. the trailing block: A_qq -= U_pq^T U_pq (FP64 MFMA tiles).
// The block's inverse then comes from the diagonal blocks' W_pp by
// recursive doubling over 16, 32 and 64: the inverse of [A B; 0 C] has the
// off-diagonal block -A^-1 (B C^-1).  W_pp waits in the lower triangle of
// its diagonal block (the diagonal in wdiag).  Positions past nb carry an
// identity (no threshold test), so they add exact zeros.  The panel wave's
// step is a short dependent chain (pivot, root, LDS round trip, FMAs); the
// panel width keeps its per-step work small, and the rest of the block runs
// on all 16 waves.
template <int SZ>
__device__ __forceinline__ void inverse_doubling_level(double (*Us)[CB + 1], int wave, int lane) {
    constexpr int ts = SZ / 16;            // tiles per side of an SZ x SZ block
    constexpr int per = ts * ts;           // tiles per pair of diagonal blocks
    constexpr int pairs = CB / (2 * SZ);
    static_assert(pairs * per <= CPT / 64, "one tile per wave");
    const bool has = wave < pairs * per;
    const int i0 = has ? 2 * SZ * (wave / per) : 0;
    const int ra = 16 * ((wave % per) / ts), cb = 16 * (wave % ts);  // tile within the block
    // T = B C^-1, staged across a barrier into B
    d4v acc = d4v{0.0, 0.0, 0.0, 0.0};
    if (has)
        acc = mma16_f64<SZ>(
            acc, lane, [&](int r, int k) { return Us[i0 + ra + r][i0 + SZ + k]; },
            [&](int k, int c) { return Us[i0 + SZ + k][i0 + SZ + cb + c]; });
    __syncthreads();
    if (has)
#pragma unroll
        for (int v = 0; v < 4; ++v) Us[i0 + ra + Mfma16<double>::row(lane, v)][i0 + SZ + cb + (lane & 15)] = acc[v];
    __syncthreads();
    // -A^-1 T, likewise
    acc = d4v{0.0, 0.0, 0.0, 0.0};
    if (has)
        acc = mma16_f64<SZ>(
            acc, lane, [&](int r, int k) { return -Us[i0 + ra + r][i0 + k]; },
            [&](int k, int c) { return Us[i0 + k][i0 + SZ + cb + c]; });
    __syncthreads();
    if (has)
#pragma unroll
        for (int v = 0; v < 4; ++v) Us[i0 + ra + Mfma16<double>::row(lane, v)][i0 + SZ + cb + (lane & 15)] = acc[v];
    __syncthreads();
}

__device__ __forceinline__ void potrf_block_body(double* __restrict__ U, int64_t ldu, int64_t k0,
                                                 int nb, double thr, double* __restrict__ W,
                                                 int64_t ldw, int* flag) {
    static_assert(CB == 128 && CPT == 1024 && PW == 16 && TS == 2, "8 panels of 16, 16 waves");
    __shared__ double Us[CB][CB + 1];
    __shared__ __attribute__((aligned(16))) double rowb[PW];
    __shared__ __attribute__((aligned(16))) double colb[PW];
    __shared__ double wdiag[CB];
    __shared__ int stop;
    if (*flag) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        double x[CB * CB / CPT];
#pragma unroll
        for (int q = 0; q < CB * CB / CPT; ++q) {  // all loads in flight, then the stores
            const int e = tid + q * CPT, i = e >> 7, c = e & (CB - 1);
            x[q] = (i < nb && c < nb && c >= i) ? U[(k0 + i) * ldu + k0 + c] : (i == c && i >= nb ? 1.0 : 0.0);
        }
#pragma unroll
        for (int q = 0; q < CB * CB / CPT; ++q) {
            const int e = tid + q * CPT;
            Us[e >> 7][e & (CB - 1)] = x[q];
        }
    }
    if (tid < CB) wdiag[tid] = 1.0;
    if (tid == 0) stop = 0;
    __syncthreads();

    for (int P0 = 0; P0 < nb; P0 += PW) {
        if (wave == 0) {
            const int rg = lane >> 3, cg = lane & 7;
            const bool act = cg >= rg;  // tiles on or above the diagonal
            double u[TS][TS], sw[TS][TS];
#pragma unroll
            for (int a = 0; a < TS; ++a)
#pragma unroll
                for (int b = 0; b < TS; ++b) {
                    const int i = TS * rg + a, c = TS * cg + b;
                    u[a][b] = (act && c >= i) ? Us[P0 + i][P0 + c] : 0.0;
                    sw[a][b] = 0.0;
                }
            // rowb needs no clearing: at step j its entries <= j hold zeros
            // (each entry's last write, at a step >= its index, is a zero);
            // colb starts the panel at zero, and its entries > j stay zero
            if (lane < PW) colb[lane] = 0.0;
            bool bad = false;
            for (int jr = 0; jr < PW / TS && !bad; ++jr) {
#pragma unroll
                for (int ja = 0; ja < TS; ++ja) {
                    const int j = TS * jr + ja;
                    const double d = readlane_f64(u[ja][ja], 9 * jr);  // lane (jr, jr)
                    const bool pad = P0 + j >= nb;                      // identity position
                    if (!pad && !(d > thr)) {
                        bad = true;
                        break;
                    }
                    const double dd = pad ? 1.0 : d;
                    // 1 / sqrt(dd): the hardware estimate (about 23 bits) and
                    // two Newton-Raphson steps y <- y (3 - dd y^2) / 2; the
                    // root is dd y
                    const double hd = 0.5 * dd;
                    double y = __builtin_amdgcn_rsq(dd);
                    y = y * fma(-hd, y * y, 1.5);
                    y = y * fma(-hd, y * y, 1.5);
                    const double rj = dd * y, inv = y;
                    if (rg == jr && act) {  // row j of U_pp; rowb gets zero at j and left of it
                        d2v x;
#pragma unroll
                        for (int b = 0; b < TS; ++b) {
                            const int c = TS * cg + b;
                            const double v = c > j ? u[ja][b] * inv : 0.0;
                            u[ja][b] = c == j ? rj : v;
                            x[b] = v;
                        }
                        *(d2v*)&rowb[TS * cg] = x;
                    }
                    if (cg == jr && act) {  // column j of W_pp (zero below j)
                        d2v x;
#pragma unroll
                        for (int a = 0; a < TS; ++a) {
                            const int i = TS * rg + a;
                            const double w = i <= j ? ((i == j ? 1.0 : 0.0) - sw[a][ja]) * inv : 0.0;
                            sw[a][ja] = w;
                            x[a] = w;
                        }
                        *(d2v*)&colb[TS * rg] = x;
                    }
                    // One wave: its LDS operations complete in order, so a
                    // wavefront-scope fence (no instruction; it keeps the
                    // compiler from moving the reads above the other lanes'
                    // writes) makes the row and column just written visible.
                    // The zeros in them leave rows <= j of U and columns
                    // <= j of W unchanged.
                    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                    const d2v ri = *(const d2v*)&rowb[TS * rg];
                    const d2v wi = *(const d2v*)&colb[TS * rg];
                    const d2v rc = *(const d2v*)&rowb[TS * cg];
#pragma unroll
                    for (int a2 = 0; a2 < TS; ++a2)
#pragma unroll
                        for (int b2 = 0; b2 < TS; ++b2) {
                            u[a2][b2] = fma(-ri[a2], rc[b2], u[a2][b2]);
                            sw[a2][b2] = fma(wi[a2], rc[b2], sw[a2][b2]);
                        }
                }
            }
            if (bad) {
                if (lane == 0) stop = 1;
            } else if (act) {
#pragma unroll
                for (int a = 0; a < TS; ++a)
#pragma unroll
                    for (int b = 0; b < TS; ++b) {
                        const int i = TS * rg + a, c = TS * cg + b;
                        if (c >= i) Us[P0 + i][P0 + c] = u[a][b];
                        if (c > i) Us[P0 + c][P0 + i] = sw[a][b];  // W_pp, transposed below
                        if (c == i) wdiag[P0 + i] = sw[a][b];
                    }
            }
        }
        __syncthreads();
        if (stop) {
            if (tid == 0) *flag = 1;  // the block leaves together
            return;
        }
        const int Q0 = P0 + PW, nq = CB - Q0;
        if (Q0 >= nb) break;  // the rest is identity
        // U_pq = W_pp^T A_pq: nq / 16 tiles, one per wave
        const int tq = nq / 16;
        d4v acc = d4v{0.0, 0.0, 0.0, 0.0};
        const bool has = wave < tq;
        if (has)
            acc = mma16_f64<PW>(
                acc, lane,
                [&](int r, int k) {  // W_pp^T (r, k) = W_pp (k, r), zero for k > r
                    const double x = Us[P0 + r][P0 + k];
                    return k < r ? x : (k == r ? wdiag[P0 + r] : 0.0);
                },
                [&](int k, int c) { return Us[P0 + k][Q0 + 16 * wave + c]; });
        __syncthreads();
        if (has)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Us[P0 + Mfma16<double>::row(lane, v)][Q0 + 16 * wave + (lane & 15)] = acc[v];
        __syncthreads();
        // A_qq -= U_pq^T U_pq on the upper tiles (tq (tq + 1) / 2 of them)
        for (int t = wave; t < tq * (tq + 1) / 2; t += CPT / 64) {
            int ta = 0, rem = t;
            while (rem >= tq - ta) {
                rem -= tq - ta;
                ++ta;
            }
            const int tb = ta + rem;  // tile (ta, tb), ta <= tb
            d4v c;
#pragma unroll
            for (int v = 0; v < 4; ++v)
                c[v] = Us[Q0 + 16 * ta + Mfma16<double>::row(lane, v)][Q0 + 16 * tb + (lane & 15)];
            c = mma16_f64<PW>(
                c, lane, [&](int r, int k) { return -Us[P0 + k][Q0 + 16 * ta + r]; },
                [&](int k, int cc) { return Us[P0 + k][Q0 + 16 * tb + cc]; });
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = 16 * ta + Mfma16<double>::row(lane, v), cc = 16 * tb + (lane & 15);
                if (cc >= r) Us[Q0 + r][Q0 + cc] = c[v];
            }
        }
        __syncthreads();
    }

    // the factor
#pragma unroll
    for (int q = 0; q < CB * CB / CPT; ++q) {
        const int e = tid + q * CPT, i = e >> 7, c = e & (CB - 1);
        if (i < nb && c < nb) U[(k0 + i) * ldu + k0 + c] = c >= i ? Us[i][c] : 0.0;
    }
    __syncthreads();  // U read out of Us before its diagonal blocks turn into W_pp
    // diagonal blocks: W_pp (upper, from the lower triangle), zero below
#pragma unroll
    for (int q = 0; q < CB * PW / CPT; ++q) {
        const int e = tid + q * CPT;
        const int P0 = PW * (e / (PW * PW)), i = (e / PW) % PW, c = e % PW;
        if (c > i) {
            const double w = Us[P0 + c][P0 + i];
            Us[P0 + c][P0 + i] = 0.0;
            Us[P0 + i][P0 + c] = w;
        } else if (c == i) {
            Us[P0 + i][P0 + i] = wdiag[P0 + i];
        }
    }
    __syncthreads();
    inverse_doubling_level<16>(Us, wave, lane);
    inverse_doubling_level<32>(Us, wave, lane);
    inverse_doubling_level<64>(Us, wave, lane);
#pragma unroll
    for (int q = 0; q < CB * CB / CPT; ++q) {
        const int e = tid + q * CPT, i = e >> 7, c = e & (CB - 1);
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

__global__ void diag_copy_kernel(int64_t n, const double* __restrict__ M, int64_t ldm,
                                 double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = M[i * ldm + i];
}

__global__ void gather_entries_kernel(int64_t count, const int64_t* __restrict__ off,
                                      const double* __restrict__ M, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = M[off[i]];
}

// eq[p] = 1 when rows a = pr[2 p] and b = pr[2 p + 1] of the symmetric M
// (upper triangle read) are bitwise equal, one block per pair
__global__ __launch_bounds__(256) void rows_equal_kernel(int64_t n, const int32_t* __restrict__ pr,
                                                         const double* __restrict__ M, int64_t ldm,
                                                         int32_t* __restrict__ eq) {
    __shared__ int differ;
    if (threadIdx.x == 0) differ = 0;
    __syncthreads();
    const int64_t a = pr[2 * blockIdx.x], b = pr[2 * blockIdx.x + 1];
    bool d = false;
    for (int64_t k = threadIdx.x; k < n; k += 256) {
        const double x = k >= a ? M[a * ldm + k] : M[k * ldm + a];
        const double y = k >= b ? M[b * ldm + k] : M[k * ldm + b];
        d |= __double_as_longlong(x) != __double_as_longlong(y);
    }
    if (d) differ = 1;  // benign race: every writer stores 1
    __syncthreads();
    if (threadIdx.x == 0) eq[blockIdx.x] = differ ? 0 : 1;
}

// U (r x r, ld ldu) = upper triangle of M[S][:, S] (M's upper triangle read),
// zero below the diagonal
__global__ void gather_upper_kernel(int64_t r, const int32_t* __restrict__ S,
                                    const double* __restrict__ M, int64_t ldm,
                                    double* __restrict__ U, int64_t ldu) {
    for (int64_t i = blockIdx.y; i < r; i += gridDim.y) {
        const int64_t si = S[i];
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < r;
             c += (int64_t)gridDim.x * blockDim.x) {
            const int64_t sc = S[c];  // S ascending: sc >= si when c >= i
            U[i * ldu + c] = c >= i ? M[si * ldm + sc] : 0.0;
        }
    }
}

// U[:, r + t] = U[:, src[t]] on rows 0 .. r - 1 (U upper triangular there)
__global__ void gather_cols_kernel(int64_t r, int64_t c, const int32_t* __restrict__ src,
                                   double* __restrict__ U, int64_t ldu) {
    for (int64_t i = blockIdx.y; i < r; i += gridDim.y)
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < c;
             t += (int64_t)gridDim.x * blockDim.x) {
            const int64_t j = src[t];
            U[i * ldu + r + t] = i <= j ? U[i * ldu + j] : 0.0;
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

void launch_diag_copy(hipStream_t s, int64_t n, const double* M, int64_t ldm, double* out) {
    if (n <= 0) return;
    diag_copy_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(n, M, ldm, out);
    ELM_LAUNCH_CHECK();
}

int64_t duplicate_nodes(hipStream_t s, int64_t n, const double* M, int64_t ldm,
                        const std::vector<double>& diag, Workspace& ws, std::vector<int32_t>& rep) {
    rep.resize((size_t)n);
    for (int64_t i = 0; i < n; ++i) rep[(size_t)i] = (int32_t)i;
    // candidate pairs: equal diagonal values, grouped by an open-addressing
    // hash of their bits (linear in n; sorting 10000 values took about a
    // millisecond of host time)
    int64_t cap = 16;
    while (cap < 2 * n) cap <<= 1;
    const int sh = 64 - __builtin_ctzll((unsigned long long)cap);
    std::vector<uint64_t> key((size_t)cap);
    std::vector<int32_t> head((size_t)cap, -1), tail((size_t)cap, -1), next((size_t)n, -1);
    std::vector<int64_t> multi;  // slots holding two or more indices
    for (int64_t i = 0; i < n; ++i) {
        uint64_t b;
        std::memcpy(&b, &diag[(size_t)i], sizeof b);
        int64_t h = (int64_t)((b * 0x9E3779B97F4A7C15ull) >> sh);
        while (head[(size_t)h] >= 0 && key[(size_t)h] != b) h = (h + 1) & (cap - 1);
        if (head[(size_t)h] < 0) {
            key[(size_t)h] = b;
            head[(size_t)h] = tail[(size_t)h] = (int32_t)i;
        } else {
            if (head[(size_t)h] == tail[(size_t)h]) multi.push_back(h);
            next[(size_t)tail[(size_t)h]] = (int32_t)i;
            tail[(size_t)h] = (int32_t)i;
        }
    }
    constexpr size_t MAX_PAIRS = 1 << 16;
    std::vector<int64_t> off;
    std::vector<int32_t> pr;
    for (int64_t h : multi) {  // each group's indices ascend along its chain
        for (int32_t i = head[(size_t)h]; i >= 0; i = next[(size_t)i])
            for (int32_t j = next[(size_t)i]; j >= 0; j = next[(size_t)j]) {
                if (off.size() >= MAX_PAIRS) return -1;  // too many equal values to check
                off.push_back((int64_t)i * ldm + j);  // the upper triangle holds the Gram
                pr.push_back(i);
                pr.push_back(j);
            }
    }
    if (off.empty()) return 0;
    // the cross terms of the candidates: M_ij = M_ii (= M_jj) marks a pair
    const int64_t cnt = (int64_t)off.size();
    int64_t* doff = (int64_t*)ws.get("dup_off", off.size() * sizeof(int64_t));
    double* dval = (double*)ws.get("dup_val", off.size() * sizeof(double));
    ELM_HIP_TRY(hipMemcpyAsync(doff, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    gather_entries_kernel<<<(unsigned)cdiv(cnt, 256), 256, 0, s>>>(cnt, doff, M, dval);
    ELM_LAUNCH_CHECK();
    std::vector<double> val(off.size());
    ELM_HIP_TRY(hipMemcpyAsync(val.data(), dval, off.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> cand;
    for (size_t k = 0; k < off.size(); ++k)
        if (val[k] == diag[(size_t)pr[2 * k]]) {
            cand.push_back(pr[2 * k]);
            cand.push_back(pr[2 * k + 1]);
        }
    if (cand.empty()) return 0;
    // and their whole rows, bitwise
    const int64_t np = (int64_t)cand.size() / 2;
    int32_t* dpr = (int32_t*)ws.get("dup_pairs", cand.size() * sizeof(int32_t));
    int32_t* deq = (int32_t*)ws.get("dup_eq", (size_t)np * sizeof(int32_t));
    ELM_HIP_TRY(hipMemcpyAsync(dpr, cand.data(), cand.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    rows_equal_kernel<<<(unsigned)np, 256, 0, s>>>(n, dpr, M, ldm, deq);
    ELM_LAUNCH_CHECK();
    std::vector<int32_t> eq((size_t)np);
    ELM_HIP_TRY(hipMemcpyAsync(eq.data(), deq, (size_t)np * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    // groups of equal rows (union-find), each represented by its lowest index
    std::function<int32_t(int32_t)> find = [&](int32_t x) {
        while (rep[(size_t)x] != x) x = rep[(size_t)x] = rep[(size_t)rep[(size_t)x]];
        return x;
    };
    for (int64_t p = 0; p < np; ++p) {
        if (!eq[(size_t)p]) continue;
        const int32_t x = find(cand[2 * p]), y = find(cand[2 * p + 1]);
        if (x != y) rep[(size_t)std::max(x, y)] = std::min(x, y);
    }
    int64_t dup = 0;
    for (int64_t i = 0; i < n; ++i) {
        rep[(size_t)i] = find((int32_t)i);
        dup += rep[(size_t)i] != i;
    }
    return dup;
}

bool dedup_cholesky(hipStream_t s, int64_t n, const double* M, int64_t ldm,
                    const std::vector<int32_t>& rep, double thr, double** R_out, elm_factor* f,
                    Workspace& ws, hipStream_t side, hipEvent_t ev_main, hipEvent_t ev_side) {
    *R_out = nullptr;
    std::vector<int32_t> S, D, pos((size_t)n, -1);
    for (int64_t j = 0; j < n; ++j)
        if (rep[(size_t)j] == j) {
            pos[(size_t)j] = (int32_t)S.size();
            S.push_back((int32_t)j);
        } else {
            D.push_back((int32_t)j);
        }
    const int64_t r = (int64_t)S.size(), c = (int64_t)D.size();
    std::vector<int32_t> src((size_t)c), piv((size_t)n);
    for (int64_t t = 0; t < c; ++t) src[(size_t)t] = pos[(size_t)rep[(size_t)D[(size_t)t]]];
    std::copy(S.begin(), S.end(), piv.begin());
    std::copy(D.begin(), D.end(), piv.begin() + r);
    int32_t* dS = (int32_t*)ws.get("dd_S", (size_t)std::max<int64_t>(r, 1) * sizeof(int32_t));
    int32_t* dsrc = (int32_t*)ws.get("dd_src", (size_t)std::max<int64_t>(c, 1) * sizeof(int32_t));
    ELM_HIP_TRY(hipMemcpyAsync(dS, S.data(), (size_t)r * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (c > 0)
        ELM_HIP_TRY(hipMemcpyAsync(dsrc, src.data(), (size_t)c * sizeof(int32_t), hipMemcpyHostToDevice, s));
    ELM_HIP_TRY(hipMemcpyAsync(f->piv, piv.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    // R = [R11 R12] (r x n, ld n) in the order S, D
    double* U = (double*)factor_alloc(f, "R", (size_t)r * n * sizeof(double));
    int* flag = (int*)ws.get("fr_flag", sizeof(int));
    clear_flag_kernel<<<1, 64, 0, s>>>(flag);
    ELM_LAUNCH_CHECK();
    gather_upper_kernel<<<dim3((unsigned)cdiv(r, 256), (unsigned)std::min<int64_t>(r, 65535)), 256, 0, s>>>(
        r, dS, M, ldm, U, n);
    ELM_LAUNCH_CHECK();
    cholesky_blocked(s, r, U, n, thr, flag, ws, side, ev_main, ev_side);
    int hflag = 0;
    ELM_HIP_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ELM_HIP_TRY(hipStreamSynchronize(s));
    if (hflag) {
        if (!f->pool) (void)hipFree(U);
        return false;
    }
    // a copy's Gram column is its original's: R12 column t = U^-T M[S, D_t] =
    // column src[t] of U
    if (c > 0) {
        gather_cols_kernel<<<dim3((unsigned)cdiv(c, 256), (unsigned)std::min<int64_t>(r, 65535)), 256, 0,
                             s>>>(r, c, dsrc, U, n);
        ELM_LAUNCH_CHECK();
    }
    *R_out = U;
    return true;
}

void launch_iota(hipStream_t s, int64_t n, int32_t* piv) {
    if (n <= 0) return;
    iota_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(n, piv);
    ELM_LAUNCH_CHECK();
}

}  // namespace elm
