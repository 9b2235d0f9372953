// General FP64 matrix product on the 16x16x4 FP64 MFMA, for the dense steps
// after the rank reveal: the block triangular inverse of R11, K = R11^-1 R12
// and the Gram I + K K^T of G.  Operands are strided views, so transposes
// cost nothing:
//   C[i][j] = alpha * sum_k A(i, k) B(k, j) + beta * C[i][j],
//   A(i, k) = A[i * a_rs + k * a_cs],  B(k, j) = B[k * b_rs + j * b_cs].
// A triangular operand can be declared so that tiles skip its zero half:
//   tri_a: A is upper triangular (A(i, k) = 0 for k < i);
//   tri_b: B is upper triangular (B(k, j) = 0 for k > j).
// The skipped products are exact zeros, so the result is the same.
// A batch of equally shaped products (blockIdx.z) shares one launch.
// upper_c: only tiles that reach the upper triangle of C (i <= j) are
// computed (a symmetric update); skip (device flag, may be NULL): the launch
// does nothing when it is set.
#include "elm_internal.h"

namespace elm {
namespace {

constexpr int BK = 16;

// TS x TS output tile, NTH / 64 waves in 2 x (NTH / 128), each (TS / 2) x
// (TS / (NTH / 128)) as blocks of 16 x 16; k-major LDS tiles, double-buffered
// through registers.  The 128-wide tile runs 8 waves (four per SIMD with two
// blocks per CU), so each wave holds 4 x 2 accumulator blocks.
template <int TS, int NTH>
__device__ __forceinline__ void gemm_body(int64_t bx, int64_t by, int64_t bz, int64_t M, int64_t N,
                                          int64_t K, double alpha, const double* __restrict__ A,
                                          int64_t a_rs, int64_t a_cs, int64_t a_bs,
                                          const double* __restrict__ B, int64_t b_rs, int64_t b_cs,
                                          int64_t b_bs, double beta, double* __restrict__ C,
                                          int64_t ldc, int64_t c_bs, int tri_a, int tri_b,
                                          int upper_c, const int* __restrict__ skip) {
    constexpr int P = TS + 16;           // LDS pitch (see the hidden-layer kernel)
    constexpr int EPT = TS * BK / NTH;   // elements per thread per operand tile
    constexpr int WGN = NTH / 128;       // waves across the tile's columns
    constexpr int WBI = TS / 32;         // 16 x 16 blocks per wave: rows
    constexpr int WBJ = TS / WGN / 16;   //                          columns
    static_assert(EPT >= 1 && WBJ >= 1, "tile and block size");
    __shared__ double As[2][BK][P];
    __shared__ double Bs[2][BK][P];
    const int64_t i0 = bx * TS, j0 = by * TS;
    if (upper_c && i0 >= j0 + TS) return;  // strictly below the diagonal
    if (skip && *skip) return;
    A += bz * a_bs;
    B += bz * b_bs;
    C += bz * c_bs;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WGN, wn = wave % WGN;
    const bool a_kcontig = (a_cs == 1);
    const bool b_jcontig = (b_cs == 1);

    // k range of this tile: triangular operands have zero blocks
    int64_t k_lo = 0, k_hi = K;
    if (tri_a) k_lo = (i0 / BK) * BK;
    if (tri_b) k_hi = (j0 + TS < K) ? j0 + TS : K;

    // thread -> EPT consecutive elements along the operand's contiguous
    // dimension: (row, k + e) for a k-contiguous A, (row + e, k) otherwise
    const int ta = tid * EPT;
    const int a_i = a_kcontig ? ta / BK : ta % TS, a_k = a_kcontig ? ta % BK : ta / TS;
    const int b_j = b_jcontig ? ta % TS : ta / BK, b_k = b_jcontig ? ta / TS : ta % BK;
    const int a_di = a_kcontig ? 0 : 1, a_dk = a_kcontig ? 1 : 0;
    const int b_dj = b_jcontig ? 1 : 0, b_dk = b_jcontig ? 0 : 1;
    double av[EPT], bv[EPT];
    // Rows past M and columns past N read clamped (in-range) addresses; their
    // results are never stored.  Only k needs masking, and only in a chunk
    // that crosses k_hi (a block-uniform branch): per-lane guarded loads would
    // compile to branches whose joins wait for each load.
    int64_t arow[EPT], bcol[EPT];
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int64_t gi = i0 + a_i + e * a_di, gj = j0 + b_j + e * b_dj;
        arow[e] = gi < M ? gi : M - 1;
        bcol[e] = gj < N ? gj : N - 1;
    }
    auto load = [&](int64_t k0) {
        if (k0 + BK <= k_hi) {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                av[e] = A[arow[e] * a_rs + (k0 + a_k + e * a_dk) * a_cs];
                bv[e] = B[(k0 + b_k + e * b_dk) * b_rs + bcol[e] * b_cs];
            }
        } else {
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int64_t gk = k0 + a_k + e * a_dk, gkb = k0 + b_k + e * b_dk;
                av[e] = gk < k_hi ? A[arow[e] * a_rs + gk * a_cs] : 0.0;
                bv[e] = gkb < k_hi ? B[gkb * b_rs + bcol[e] * b_cs] : 0.0;
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < EPT; ++e) {
            As[buf][a_k + e * a_dk][a_i + e * a_di] = av[e];
            Bs[buf][b_k + e * b_dk][b_j + e * b_dj] = bv[e];
        }
    };

    d4v acc[WBI][WBJ];
#pragma unroll
    for (int x = 0; x < WBI; ++x)
#pragma unroll
        for (int y = 0; y < WBJ; ++y) acc[x][y] = d4v{};

    if (k_lo < k_hi) {
        load(k_lo);
        store(0);
        __syncthreads();
        int buf = 0;
        for (int64_t k0 = k_lo; k0 < k_hi; k0 += BK) {
            const bool more = k0 + BK < k_hi;
            if (more) load(k0 + BK);
#pragma unroll
            for (int kk = 0; kk < BK; kk += 4) {
                const int k = kk + (lane >> 4);
                double a[WBI], b[WBJ];
#pragma unroll
                for (int x = 0; x < WBI; ++x) a[x] = As[buf][k][wm * (TS / 2) + x * 16 + (lane & 15)];
#pragma unroll
                for (int y = 0; y < WBJ; ++y)
                    b[y] = Bs[buf][k][wn * (TS / WGN) + y * 16 + (lane & 15)];
#pragma unroll
                for (int x = 0; x < WBI; ++x)
#pragma unroll
                    for (int y = 0; y < WBJ; ++y) acc[x][y] = Mfma16<double>::op(a[x], b[y], acc[x][y]);
            }
            if (more) store(buf ^ 1);
            __syncthreads();
            buf ^= 1;
        }
    }
    // With beta != 0 a block row's C values are read together (clamped
    // addresses, all in range) before its stores: read, wait and store per
    // element had put 32 memory round trips after every tile.
    const bool use_c = beta != 0.0;  // block-uniform
#pragma unroll
    for (int x = 0; x < WBI; ++x) {
        double cold[WBJ][4];
        if (use_c) {
#pragma unroll
            for (int y = 0; y < WBJ; ++y)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t gi = i0 + wm * (TS / 2) + x * 16 + Mfma16<double>::row(lane, v);
                    const int64_t gj = j0 + wn * (TS / WGN) + y * 16 + (lane & 15);
                    cold[y][v] = C[(gi < M ? gi : M - 1) * ldc + (gj < N ? gj : N - 1)];
                }
        }
#pragma unroll
        for (int y = 0; y < WBJ; ++y)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = i0 + wm * (TS / 2) + x * 16 + Mfma16<double>::row(lane, v);
                const int64_t gj = j0 + wn * (TS / WGN) + y * 16 + (lane & 15);
                if (gi >= M || gj >= N) continue;
                double c = alpha * acc[x][y][v];
                if (use_c) c += beta * cold[y][v];
                C[gi * ldc + gj] = c;
            }
    }
}

template <int TS, int NTH>
__global__ __launch_bounds__(NTH, NTH / 128) void gemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                     const double* __restrict__ A, int64_t a_rs,
                                                     int64_t a_cs, int64_t a_bs,
                                                     const double* __restrict__ B, int64_t b_rs,
                                                     int64_t b_cs, int64_t b_bs, double beta,
                                                     double* __restrict__ C, int64_t ldc,
                                                     int64_t c_bs, int tri_a, int tri_b, int upper_c,
                                                     const int* __restrict__ skip) {
    // A triangular operand makes the tiles' k ranges unequal: blocks are
    // dispatched in the order of their ids, so the longest tiles take the
    // first ids (tri_a: the top tile rows first; tri_b: the rightmost tile
    // columns first) and the short ones fill in behind them.
    int64_t bx = blockIdx.x, by = blockIdx.y;
    if (tri_a || tri_b) {
        const int64_t b = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
        if (tri_a) {
            bx = b / gridDim.y;
            by = b % gridDim.y;
        } else {
            by = gridDim.y - 1 - b / gridDim.x;
            bx = b % gridDim.x;
        }
    }
    gemm_body<TS, NTH>(bx, by, blockIdx.z, M, N, K, alpha, A, a_rs, a_cs, a_bs, B, b_rs, b_cs, b_bs,
                       beta, C, ldc, c_bs, tri_a, tri_b, upper_c, skip);
}

// products of a grouped launch: blocks of a descriptor run over its tiles
// (rows fastest, then columns, then the batch)
template <int TS, int NTH>
__global__ __launch_bounds__(NTH, NTH / 128) void gemm_grouped(const GemmDesc* __restrict__ d,
                                                               GroupSched g) {
    int64_t lb;
    const GemmDesc& q = d[group_problem(g, lb)];
    const int64_t nx = cdiv(q.M, TS), ny = cdiv(q.N, TS);
    const int64_t bx = lb % nx, t = lb / nx;
    gemm_body<TS, NTH>(bx, t % ny, t / ny, q.M, q.N, q.K, q.alpha, q.A, q.a_rs, q.a_cs, q.a_bs, q.B,
                       q.b_rs, q.b_cs, q.b_bs, q.beta, q.C, q.ldc, q.c_bs, q.tri_a, q.tri_b, 0,
                       nullptr);
}

}  // namespace

// 128-wide tiles when there are enough of them to give every CU one;
// otherwise (thin strips of the blocked factorisations) four times as many
// 64-wide tiles.  With a triangular operand the tiles' k ranges run from one
// chunk to the whole K, so a launch of fewer than 768 128-wide tiles (a round
// and a half at two per CU) lasts as long as its longest tiles while the
// others' CUs idle: such products also take 64-wide tiles, whose shorter
// tiles fill the rounds (the triangular inverse's levels of order 1024 and
// 2048 at L = 10000: 8.7 -> 8.2 ms per factor step; 1536 measured the same).
static bool use_tile128(int64_t batch, int64_t M, int64_t N, bool tri) {
    const int64_t t = cdiv(M, 128) * cdiv(N, 128) * batch;
    return M >= 128 && N >= 128 && t >= 256 && !(tri && t < 768);
}

int gemm_tile(const GemmDesc& q) {
    return use_tile128(q.batch, q.M, q.N, q.tri_a || q.tri_b) ? 128 : 64;
}

int64_t gemm_group_blocks(const GemmDesc& q, int ts) {
    if (q.M <= 0 || q.N <= 0 || q.batch <= 0) return 0;
    return cdiv(q.M, ts) * cdiv(q.N, ts) * q.batch;
}

void launch_gemm_grouped(hipStream_t s, int ts, const GemmDesc* d, const GroupSched& g) {
    if (g.count <= 0 || g.blocks <= 0) return;
    if (ts == 128)
        gemm_grouped<128, 512><<<(unsigned)g.blocks, 512, 0, s>>>(d, g);
    else
        gemm_grouped<64, 256><<<(unsigned)g.blocks, 256, 0, s>>>(d, g);
    ELM_LAUNCH_CHECK();
}

void gemm_f64_batched(hipStream_t s, int64_t batch, int64_t M, int64_t N, int64_t K, double alpha,
                      const double* A, int64_t a_rs, int64_t a_cs, int64_t a_bs, const double* B,
                      int64_t b_rs, int64_t b_cs, int64_t b_bs, double beta, double* C, int64_t ldc,
                      int64_t c_bs, bool tri_a, bool tri_b, bool upper_c, const int* skip) {
    if (M <= 0 || N <= 0 || batch <= 0) return;
    if (use_tile128(batch, M, N, tri_a || tri_b)) {  // the rule of gemm_tile
        dim3 grid((unsigned)cdiv(M, 128), (unsigned)cdiv(N, 128), (unsigned)batch);
        gemm_kernel<128, 512><<<grid, 512, 0, s>>>(M, N, K, alpha, A, a_rs, a_cs, a_bs, B, b_rs, b_cs,
                                                   b_bs, beta, C, ldc, c_bs, tri_a, tri_b, upper_c, skip);
    } else {
        dim3 grid((unsigned)cdiv(M, 64), (unsigned)cdiv(N, 64), (unsigned)batch);
        gemm_kernel<64, 256><<<grid, 256, 0, s>>>(M, N, K, alpha, A, a_rs, a_cs, a_bs, B, b_rs, b_cs,
                                                  b_bs, beta, C, ldc, c_bs, tri_a, tri_b, upper_c, skip);
    }
    ELM_LAUNCH_CHECK();
}

void gemm_f64(hipStream_t s, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
              int64_t a_rs, int64_t a_cs, const double* B, int64_t b_rs, int64_t b_cs, double beta,
              double* C, int64_t ldc) {
    gemm_f64_batched(s, 1, M, N, K, alpha, A, a_rs, a_cs, 0, B, b_rs, b_cs, 0, beta, C, ldc, 0, false,
                     false);
}

}  // namespace elm
